/*
 * A plain C program that uses libmassivemds through its C ABI alone (no
 * Python, no torch): the boundary of include/massivemds.h is self-contained.
 *
 *   capi_roundtrip cpu                 host-only entry points and rejects
 *   capi_roundtrip gpu IN.bin OUT.bin  one fused evaluation on the device
 *
 * IN.bin: int64 n, int32 d, int32 pad, double sigma, then x (n*d doubles,
 * row-major) and y (n*n doubles, row-major; NaN = missing).  OUT.bin: double
 * loglik, double dsigma, int64 m_obs, then the gradient (n*d doubles).
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "massivemds.h"

#define CHECK(cond, msg)                                            \
    do {                                                            \
        if (!(cond)) {                                              \
            fprintf(stderr, "FAILED: %s (%s)\n", msg, mds_last_error()); \
            return 1;                                               \
        }                                                           \
    } while (0)

static int host_checks(void)
{
    size_t ws = 0;
    int32_t br = 0, w = 0;
    CHECK(mds_version() > 0, "version");
    CHECK(mds_workspace_bytes(5392, 2, MDS_F64, 0, 0, &ws) == MDS_OK && ws > 0, "workspace");
    CHECK(mds_resolve_tiling(5392, 2, MDS_F64, 0, 0, &br, &w) == MDS_OK && br > 0 && w > 0,
          "resolve tiling");
    CHECK(mds_workspace_bytes(10, 9, MDS_F64, 0, 0, &ws) == MDS_ERR_UNSUPPORTED, "d > max");
    CHECK(mds_workspace_bytes(10, 2, MDS_F64, 48, 0, &ws) == MDS_ERR_UNSUPPORTED, "bad tile");
    CHECK(mds_loglik(10, 2, NULL, 2, NULL, MDS_F64, 10, NULL, NULL, NULL, 0, 0, 0, NULL) ==
              MDS_ERR_INVALID_ARGUMENT,
          "null pointers");
    CHECK(strcmp(mds_status_string(MDS_ERR_HIP), "MDS_ERR_HIP") == 0, "status string");
    CHECK(mds_require_symmetric(NULL, MDS_F64, 10, 10, NULL, NULL) == MDS_ERR_INVALID_ARGUMENT,
          "checked mode rejects NULL");
    CHECK(strcmp(mds_status_string(MDS_ERR_NOT_SYMMETRIC), "MDS_ERR_NOT_SYMMETRIC") == 0,
          "status string (symmetry)");
    printf("capi host checks ok (default tiles %dx%d, workspace %zu B at N=5392)\n", br, 64 * w,
           ws);
    return 0;
}

static int device_eval(const char* in_path, const char* out_path)
{
    FILE* f = fopen(in_path, "rb");
    CHECK(f != NULL, "open input");
    int64_t n;
    int32_t d, pad;
    double sigma;
    CHECK(fread(&n, 8, 1, f) == 1 && fread(&d, 4, 1, f) == 1 && fread(&pad, 4, 1, f) == 1 &&
              fread(&sigma, 8, 1, f) == 1,
          "read header");
    CHECK(n > 1 && n <= 8192 && d >= 1 && d <= MDS_MAX_DIM, "header values");
    double* x = (double*)malloc(sizeof(double) * (size_t)(n * d));
    double* y = (double*)malloc(sizeof(double) * (size_t)(n * n));
    double* g = (double*)malloc(sizeof(double) * (size_t)(n * d));
    CHECK(x && y && g, "host allocation");
    CHECK(fread(x, 8, (size_t)(n * d), f) == (size_t)(n * d) &&
              fread(y, 8, (size_t)(n * n), f) == (size_t)(n * n),
          "read arrays");
    fclose(f);

    const int64_t ldy = (n + 63) / 64 * 64;
    size_t wsb = 0;
    CHECK(mds_workspace_bytes(n, d, MDS_F64, 0, 0, &wsb) == MDS_OK, "workspace size");
    double *dx, *dy_src, *dy, *dg, *dsig, *dl, *dds;
    int64_t* dm;
    void* dws;
    CHECK(hipMalloc((void**)&dx, sizeof(double) * (size_t)(n * d)) == hipSuccess &&
              hipMalloc((void**)&dy_src, sizeof(double) * (size_t)(n * n)) == hipSuccess &&
              hipMalloc((void**)&dy, sizeof(double) * (size_t)(n * ldy)) == hipSuccess &&
              hipMalloc((void**)&dg, sizeof(double) * (size_t)(n * d)) == hipSuccess &&
              hipMalloc((void**)&dsig, 8) == hipSuccess && hipMalloc((void**)&dl, 8) == hipSuccess &&
              hipMalloc((void**)&dds, 8) == hipSuccess && hipMalloc((void**)&dm, 8) == hipSuccess &&
              hipMalloc(&dws, wsb) == hipSuccess,
          "device allocation");
    CHECK(hipMemcpy(dx, x, sizeof(double) * (size_t)(n * d), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(dy_src, y, sizeof(double) * (size_t)(n * n), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(dsig, &sigma, 8, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemset(dm, 0, 8) == hipSuccess,
          "upload");
    CHECK(mds_prepare_y(dy_src, MDS_F64, n, NULL, 0, dy, MDS_F64, ldy, n, NULL, (int64_t*)dm,
                        NULL) == MDS_OK,
          "prepare");
    /* the checked mode: the prepared Y is symmetric */
    int64_t* dbad;
    CHECK(hipMalloc((void**)&dbad, 8) == hipSuccess, "device allocation (count)");
    CHECK(mds_require_symmetric(dy, MDS_F64, ldy, n, dbad, NULL) == MDS_OK, "symmetric Y accepted");
    /* Y and the prepared copy are exact-size allocations (n x n and n x ldy
       doubles): the sweep reads no row past the last one */
    CHECK(mds_gradient(n, d, dx, d, dy, MDS_F64, ldy, dsig, NULL, dg, d, dl, dds, NULL, dws, wsb,
                       0, 0, NULL) == MDS_OK,
          "gradient");
    CHECK(hipDeviceSynchronize() == hipSuccess, "synchronize");
    double L, ds;
    int64_t m;
    CHECK(hipMemcpy(g, dg, sizeof(double) * (size_t)(n * d), hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(&L, dl, 8, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(&ds, dds, 8, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(&m, dm, 8, hipMemcpyDeviceToHost) == hipSuccess,
          "download");

    /* held-out predictive density over two draws (x, and x + 0.01), one
       pass: pairs with (i + j) % 7 == 0 held out */
    uint8_t* held = (uint8_t*)malloc((size_t)(n * n));
    double* xs = (double*)malloc(sizeof(double) * (size_t)(2 * n * d));
    CHECK(held && xs, "host allocation (held-out)");
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) held[i * n + j] = (uint8_t)((i + j) % 7 == 0);
    for (int64_t k = 0; k < n * d; ++k) {
        xs[k] = x[k];
        xs[n * d + k] = x[k] + 0.01;
    }
    const double sigmas[2] = {sigma, 1.1 * sigma};
    size_t hwb = 0, fwb = 0;
    CHECK(mds_heldout_workspace_bytes(n, &hwb) == MDS_OK, "held-out workspace size");
    uint8_t* dheld;
    double *dxs, *dsigs, *dlpd;
    int64_t* dmh;
    void* dhw;
    CHECK(hipMalloc((void**)&dheld, (size_t)(n * n)) == hipSuccess &&
              hipMalloc((void**)&dxs, sizeof(double) * (size_t)(2 * n * d)) == hipSuccess &&
              hipMalloc((void**)&dsigs, 16) == hipSuccess &&
              hipMalloc((void**)&dlpd, 8) == hipSuccess && hipMalloc((void**)&dmh, 8) == hipSuccess &&
              hipMalloc(&dhw, hwb) == hipSuccess,
          "device allocation (held-out)");
    CHECK(hipMemcpy(dheld, held, (size_t)(n * n), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(dxs, xs, sizeof(double) * (size_t)(2 * n * d), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(dsigs, sigmas, 16, hipMemcpyHostToDevice) == hipSuccess,
          "upload (held-out)");
    CHECK(mds_heldout_count(dy_src, MDS_F64, n, NULL, 0, dheld, n, n, dmh, dhw, hwb, NULL) ==
              MDS_OK,
          "held-out count");
    int64_t mh = 0;
    CHECK(hipMemcpy(&mh, dmh, 8, hipMemcpyDeviceToHost) == hipSuccess && mh > 0, "held-out m");
    int32_t *dpi, *dpj;
    double *dpy, *dacc;
    void* dfw;
    CHECK(mds_lpd_workspace_bytes(mh, &fwb) == MDS_OK, "lpd workspace size");
    CHECK(hipMalloc((void**)&dpi, 4 * (size_t)mh) == hipSuccess &&
              hipMalloc((void**)&dpj, 4 * (size_t)mh) == hipSuccess &&
              hipMalloc((void**)&dpy, 8 * (size_t)mh) == hipSuccess &&
              hipMalloc((void**)&dacc, 16 * (size_t)mh) == hipSuccess &&
              hipMalloc(&dfw, fwb) == hipSuccess,
          "device allocation (pairs)");
    CHECK(mds_heldout_fill(dy_src, MDS_F64, n, NULL, 0, dheld, n, n, dhw, hwb, mh, dpi, dpj, dpy,
                           NULL) == MDS_OK,
          "held-out fill");
    CHECK(mds_lpd_accumulate_draws(mh, dpi, dpj, dpy, d, dxs, d, n * d, dsigs, 2, dacc, 1,
                                   NULL) == MDS_OK,
          "lpd accumulate (two draws)");
    CHECK(mds_lpd_finalize(mh, dacc, 2, dfw, fwb, dlpd, NULL) == MDS_OK, "lpd finalize");
    double lpd;
    CHECK(hipMemcpy(&lpd, dlpd, 8, hipMemcpyDeviceToHost) == hipSuccess, "download lpd");

    /* one pair changed on one side only: the checked mode reports it */
    int64_t ip = 1;
    while (ip < n - 1 && y[ip * n] != y[ip * n]) ++ip; /* an observed pair (ip, 0) */
    const double bump = y[ip * n] + 1.0;
    CHECK(hipMemcpy(dy + ip * ldy, &bump, 8, hipMemcpyHostToDevice) == hipSuccess, "perturb");
    CHECK(mds_require_symmetric(dy, MDS_F64, ldy, n, dbad, NULL) == MDS_ERR_NOT_SYMMETRIC,
          "asymmetric Y rejected");
    int64_t nbad = 0;
    CHECK(hipMemcpy(&nbad, dbad, 8, hipMemcpyDeviceToHost) == hipSuccess && nbad == 1,
          "one mismatched pair");
    hipFree(dbad);

    FILE* o = fopen(out_path, "wb");
    CHECK(o != NULL, "open output");
    fwrite(&L, 8, 1, o);
    fwrite(&ds, 8, 1, o);
    fwrite(&m, 8, 1, o);
    fwrite(g, 8, (size_t)(n * d), o);
    fwrite(&lpd, 8, 1, o);
    fwrite(&mh, 8, 1, o);
    fclose(o);
    hipFree(dheld);
    hipFree(dxs);
    hipFree(dsigs);
    hipFree(dlpd);
    hipFree(dmh);
    hipFree(dhw);
    hipFree(dpi);
    hipFree(dpj);
    hipFree(dpy);
    hipFree(dacc);
    hipFree(dfw);
    free(held);
    free(xs);
    hipFree(dx);
    hipFree(dy_src);
    hipFree(dy);
    hipFree(dg);
    hipFree(dsig);
    hipFree(dl);
    hipFree(dds);
    hipFree(dm);
    hipFree(dws);
    free(x);
    free(y);
    free(g);
    printf("capi device evaluation ok: n=%lld L=%.17g lpd=%.17g over %lld held-out pairs\n",
           (long long)n, L, lpd, (long long)mh);
    return 0;
}

int main(int argc, char** argv)
{
    if (argc >= 2 && strcmp(argv[1], "cpu") == 0) return host_checks();
    if (argc >= 4 && strcmp(argv[1], "gpu") == 0) return device_eval(argv[2], argv[3]);
    fprintf(stderr, "usage: %s cpu | gpu IN.bin OUT.bin\n", argv[0]);
    return 2;
}
