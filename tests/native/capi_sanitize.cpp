// The C-ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
// (no GPU): argument validation, tiling resolution, workspace and batch
// layout arithmetic and the error-message formatting of every entry point,
// over a grid of valid and invalid arguments.  Only calls that return before
// any HIP call are made (the validation runs first by contract), so no
// device is needed.  Exit status 0 and "ok" when every expectation holds and
// no sanitizer fires.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "massivemds.h"

static int g_fail = 0;
static long g_calls = 0;

#define EXPECT(cond)                                                                \
    do {                                                                            \
        ++g_calls;                                                                  \
        if (!(cond)) {                                                              \
            std::fprintf(stderr, "FAIL line %d: %s (%s)\n", __LINE__, #cond, mds_last_error()); \
            ++g_fail;                                                               \
        }                                                                           \
    } while (0)

// aligned fake device addresses: validation never dereferences them
static void* fake(uintptr_t off = 0) { return reinterpret_cast<void*>(uintptr_t(1) << 40 | off); }
static double* fd(uintptr_t off = 0) { return static_cast<double*>(fake(off)); }

static bool is_status(int s)
{
    return s == MDS_OK || s == MDS_ERR_INVALID_ARGUMENT || s == MDS_ERR_UNSUPPORTED ||
           s == MDS_ERR_WORKSPACE_TOO_SMALL;
}

static void tiling_grid()
{
    const int64_t ns[] = {-1, 0, 1, 2, 7, 63, 64, 65, 1000, 1537, 5392, 100000, MDS_MAX_N,
                          MDS_MAX_N + 1};
    const int ds[] = {0, 1, 2, 3, 4, 6, 8, 9};
    const int dts[] = {MDS_F64, MDS_F32, 2, MDS_F64 | MDS_UNTRUNCATED, MDS_F32 | 0x200};
    const int rows[] = {0, 7, 8, 16, 32, 64, 128, 256, 512};
    const int waves[] = {0, 1, 2, 3, 4, 8, 16, MDS_TILE_WAVES(1, 2), MDS_TILE_WAVES(1, 8),
                         MDS_TILE_WAVES(2, 4), MDS_TILE_WAVES(4, 4), MDS_TILE_WAVES(1, 3),
                         MDS_TILE_WAVES(0, 2), 0x10000, -1};
    for (int64_t n : ns)
        for (int d : ds)
            for (int dt : dts)
                for (int br : rows)
                    for (int tw : waves) {
                        size_t ws = 0, hws = 0;
                        int32_t r = -1, w = -1;
                        const int s1 = mds_workspace_bytes(n, d, dt, br, tw, &ws);
                        const int s2 = mds_resolve_tiling(n, d, dt, br, tw, &r, &w);
                        const int s3 = mds_hmc_workspace_bytes(n, d, dt, br, tw, &hws);
                        EXPECT(is_status(s1) && is_status(s2) && is_status(s3));
                        EXPECT(s1 == s2 && s1 == s3);
                        if (s1 == MDS_OK) {
                            EXPECT(ws % MDS_WORKSPACE_ALIGN == 0 && hws >= ws);
                            EXPECT(r >= 8 && r <= 256 && (w & 0xFF) >= 1 && (w & 0xFF) <= 8);
                            // the resolved tiling is accepted again as given
                            size_t ws2 = 0;
                            EXPECT(mds_workspace_bytes(n, d, dt, r, w, &ws2) == MDS_OK && ws2 == ws);
                        }
                        EXPECT(mds_workspace_bytes(n, d, dt, br, tw, nullptr) != MDS_OK);
                    }
}

static void entry_point_rejects()
{
    size_t ws = 0;
    EXPECT(mds_workspace_bytes(100, 2, MDS_F64, 0, 0, &ws) == MDS_OK);
    void* W = fake(0x100000);
    // loglik: NULL x, bad ldx, bad ldy, NULL sigma, misaligned y, small workspace, NULL out
    EXPECT(mds_loglik(100, 2, nullptr, 2, fake(), MDS_F64, 128, fd(), fd(), W, ws, 0, 0, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_loglik(100, 2, fd(), 1, fake(), MDS_F64, 128, fd(), fd(), W, ws, 0, 0, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_loglik(100, 2, fd(), 2, fake(), MDS_F64, 99, fd(), fd(), W, ws, 0, 0, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_loglik(100, 2, fd(), 2, fake(), MDS_F64, 128, nullptr, fd(), W, ws, 0, 0, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_loglik(100, 2, fd(), 2, fake(4), MDS_F64, 128, fd(), fd(), W, ws, 0, 0, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_loglik(100, 2, fd(), 2, fake(), MDS_F64, 128, fd(), fd(), W, ws - 1, 0, 0, nullptr) ==
           MDS_ERR_WORKSPACE_TOO_SMALL);
    EXPECT(mds_loglik(100, 2, fd(), 2, fake(), MDS_F64, 128, fd(), nullptr, W, ws, 0, 0, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_loglik(100, 2, fd(), 2, fake(), MDS_F64, 128, fd(), fd(), fake(8), ws, 0, 0,
                      nullptr) == MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_loglik(100, 2, fd(), 2, fake(), MDS_F64 | 0x400, 128, fd(), fd(), W, ws, 0, 0,
                      nullptr) == MDS_ERR_UNSUPPORTED);
    // gradient: NULL grad, ldg < d, misaligned dsigma
    EXPECT(mds_gradient(100, 2, fd(), 2, fake(), MDS_F64, 128, fd(), nullptr, nullptr, 2, nullptr,
                        nullptr, nullptr, W, ws, 0, 0, nullptr) == MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_gradient(100, 2, fd(), 2, fake(), MDS_F64, 128, fd(), nullptr, fd(), 1, nullptr,
                        nullptr, nullptr, W, ws, 0, 0, nullptr) == MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_gradient(100, 2, fd(), 2, fake(), MDS_F64, 128, fd(), nullptr, fd(), 2, nullptr,
                        fd(3), nullptr, W, ws, 0, 0, nullptr) == MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_gradient(100, 2, fd(), 2, fake(), MDS_F64, 128, fd(), nullptr, fd(), 2, nullptr,
                        nullptr, nullptr, W, ws, 48, 0, nullptr) == MDS_ERR_UNSUPPORTED);
    // leapfrog: aliasing, negative steps, NULL step
    EXPECT(mds_leapfrog(100, 2, fd(), 2, fd(), 2, fake(), MDS_F64, 128, fd(), nullptr, fd(), nullptr,
                        5, fd(0x1000), fd(), 0, nullptr, nullptr, W, ws, 0, 0, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_leapfrog(100, 2, fd(), 2, fd(0x1000), 2, fake(), MDS_F64, 128, fd(), nullptr, fd(),
                        nullptr, -1, fd(0x2000), fd(), 0, nullptr, nullptr, W, ws, 0, 0, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_leapfrog(100, 2, fd(), 2, fd(0x1000), 2, fake(), MDS_F64, 128, fd(), nullptr, nullptr,
                        nullptr, 5, fd(0x2000), fd(), 0, nullptr, nullptr, W, ws, 0, 0, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    // hmc: small workspace (the gradient workspace is not enough)
    uint64_t* it = static_cast<uint64_t*>(fake(0x3000));
    EXPECT(mds_hmc_step(100, 2, fd(), 2, fake(), MDS_F64, 128, fd(), nullptr, fd(), nullptr, 5, 1, it,
                        fd(0x1000), 2, fd(0x2000), fd(), 0, nullptr, nullptr, W, ws, 0, 0,
                        nullptr) == MDS_ERR_WORKSPACE_TOO_SMALL);
    EXPECT(mds_hmc_momentum(100, 2, nullptr, 1, nullptr, fd(), 2, nullptr) == MDS_ERR_INVALID_ARGUMENT);
    // prepare, symmetry, order, permute
    EXPECT(mds_prepare_y(fake(), MDS_F64, 99, nullptr, 0, fake(), MDS_F64, 100, 100, nullptr, nullptr,
                         nullptr) == MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_prepare_y(fake(), MDS_F64, 100, nullptr, 0, fake(), MDS_F32, 100, 100, nullptr,
                         nullptr, nullptr) == MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_check_symmetric(fake(), 5, 100, 100, static_cast<int64_t*>(fake()), nullptr) ==
           MDS_ERR_UNSUPPORTED);
    EXPECT(mds_require_symmetric(fake(), MDS_F64, 99, 100, static_cast<int64_t*>(fake()), nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    size_t ows = 0;
    EXPECT(mds_order_workspace_bytes(100, &ows) == MDS_OK && ows > 0);
    EXPECT(mds_spatial_order(100, 2, fd(), 2, static_cast<int64_t*>(fake()), W, ows - 1, nullptr) ==
           MDS_ERR_WORKSPACE_TOO_SMALL);
    EXPECT(mds_permute_rows(100, 2, fd(), 2, fd(), 2, static_cast<int64_t*>(fake()), 0, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    // held-out pairs and lpd
    size_t hws = 0, lws = 0;
    EXPECT(mds_heldout_workspace_bytes(100, &hws) == MDS_OK && hws > 0);
    EXPECT(mds_heldout_count(fake(), MDS_F64, 100, nullptr, 0, static_cast<uint8_t*>(fake()), 100,
                             100, static_cast<int64_t*>(fake()), W, hws - 1, nullptr) ==
           MDS_ERR_WORKSPACE_TOO_SMALL);
    EXPECT(mds_heldout_fill(fake(), MDS_F64, 100, nullptr, 0, static_cast<uint8_t*>(fake()), 100,
                            100, W, hws, -1, nullptr, nullptr, nullptr, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_lpd_accumulate(10, nullptr, nullptr, nullptr, 2, fd(), 2, fd(), fd(), 1, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_lpd_accumulate_draws(10, static_cast<int32_t*>(fake()), static_cast<int32_t*>(fake()),
                                    fd(), 2, fd(), 2, -1, fd(), 2, fd(), 1, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_lpd_workspace_bytes(10, &lws) == MDS_OK && lws > 0);
    EXPECT(mds_lpd_finalize(10, fd(), 0, W, lws, fd(), nullptr) == MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_log_phi(fd(), fd(), fd(), -1, MDS_F64, nullptr) == MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_log_phi(fd(), fd(), fd(), 10, 7, nullptr) == MDS_ERR_UNSUPPORTED);
    EXPECT(mds_set_sweep_events(reinterpret_cast<hipEvent_t>(fake()), nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_set_tile_trace(fake(4)) == MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_set_tile_trace(nullptr) == MDS_OK);
}

static void batch_layouts()
{
    // host descriptor tables of uneven problems: sizes and validation only
    std::vector<mds_problem_desc> ds;
    const int64_t ns[] = {0, 1, 2, 65, 500, 777, 8000};
    for (int k = 0; k < 7; ++k)
        for (int d : {1, 2, 4, 6, 8}) {
            mds_problem_desc q;
            std::memset(&q, 0, sizeof q);
            q.n = ns[k];
            q.d = d;
            q.tile_rows = (k % 3 == 0) ? 0 : (k % 3 == 1 ? 64 : 256);
            q.x = fd(0x10000 * (uintptr_t)(k + 1));
            q.ldx = d;
            q.y = fake(0x80000);
            q.ldy = (ns[k] + 63) / 64 * 64 + 64;
            q.sigma = fd(0x200);
            q.grad = fd(0x400000);
            q.ldg = d;
            ds.push_back(q);
        }
    for (int tw : {0, 1, 2, 4, 8, MDS_TILE_WAVES(1, 4), MDS_TILE_WAVES(2, 2), 3}) {
        for (int dt : {(int)MDS_F64, (int)MDS_F32, (int)MDS_F32 | MDS_UNTRUNCATED}) {
            size_t b = 0;
            const int s = mds_batch_workspace_bytes(ds.data(), (int32_t)ds.size(), dt, tw, &b);
            EXPECT(is_status(s));
            if (s == MDS_OK) EXPECT(b > 0 && b % MDS_WORKSPACE_ALIGN == 0);
        }
    }
    size_t b = 0;
    EXPECT(mds_batch_workspace_bytes(ds.data(), 0, MDS_F64, 0, &b) == MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_batch_workspace_bytes(nullptr, 3, MDS_F64, 0, &b) == MDS_ERR_INVALID_ARGUMENT);
    ds[3].ldg = 0;  // grad with ldg < d
    EXPECT(mds_batch_workspace_bytes(ds.data(), (int32_t)ds.size(), MDS_F64, 0, &b) ==
           MDS_ERR_INVALID_ARGUMENT);
    // a long error message (problem index and nested detail) stays in bounds
    EXPECT(std::strlen(mds_last_error()) < 512);
    mds_batch_plan plan;
    std::memset(&plan, 0, sizeof plan);
    EXPECT(mds_batch_eval(&plan, 1, nullptr) == MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_batch_leapfrog(&plan, 5, 0, nullptr) == MDS_ERR_INVALID_ARGUMENT);
    EXPECT(mds_batch_init(ds.data(), 1, MDS_F64, 0, nullptr, 0, nullptr, nullptr) ==
           MDS_ERR_INVALID_ARGUMENT);
}

int main()
{
    for (int s = 1; s >= -6; --s) EXPECT(mds_status_string(s) != nullptr);
    EXPECT(mds_version() > 0);
    tiling_grid();
    entry_point_rejects();
    batch_layouts();
    if (g_fail) {
        std::fprintf(stderr, "%d of %ld expectations failed\n", g_fail, g_calls);
        return 1;
    }
    std::printf("capi host code ok under sanitizers: %ld calls\n", g_calls);
    return 0;
}
