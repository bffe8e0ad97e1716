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
    CHECK(n > 1 && n <= 4096 && d >= 1 && d <= MDS_MAX_DIM, "header values");
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
    FILE* o = fopen(out_path, "wb");
    CHECK(o != NULL, "open output");
    fwrite(&L, 8, 1, o);
    fwrite(&ds, 8, 1, o);
    fwrite(&m, 8, 1, o);
    fwrite(g, 8, (size_t)(n * d), o);
    fclose(o);
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
    printf("capi device evaluation ok: n=%lld L=%.17g\n", (long long)n, L);
    return 0;
}

int main(int argc, char** argv)
{
    if (argc >= 2 && strcmp(argv[1], "cpu") == 0) return host_checks();
    if (argc >= 4 && strcmp(argv[1], "gpu") == 0) return device_eval(argv[2], argv[3]);
    fprintf(stderr, "usage: %s cpu | gpu IN.bin OUT.bin\n", argv[0]);
    return 2;
}
