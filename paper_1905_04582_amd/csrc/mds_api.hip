// mds_api.hip -- host side of the C-ABI declared in include/massivemds.h:
// argument validation (always before any HIP call), tiling defaults,
// workspace carving and the launch sequences of each entry point.
#include <stdarg.h>
#include <stdio.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/massivemds.h"
#include "mds_internal.h"

namespace mds {
hipError_t launch_kick_drift(int64_t n, int d, double* x, int64_t ldx, double* p, int64_t ldp,
                             const double* g, const double* inv_mass, const double* step,
                             double mult, int drift, hipStream_t s);
hipError_t launch_energy(int64_t n, int d, const double* x, int64_t ldx, const double* p,
                         int64_t ldp, const double* inv_mass, const double* prior,
                         const double* loglik, double* out, hipStream_t s);
hipError_t launch_prepare(const void* src, int sdt, int64_t ld_src, const uint8_t* mask,
                          int64_t ld_mask, void* out, int odt, int64_t ldy, int64_t n,
                          const int64_t* perm, int64_t* count, hipStream_t s);
size_t order_workspace_bytes(int64_t n);
hipError_t launch_order(int64_t n, int d, const double* x, int64_t ldx, int64_t* perm, void* ws,
                        hipStream_t s);
hipError_t launch_permute_rows(int64_t n, int d, const double* src, int64_t ld_src, double* dst,
                               int64_t ld_dst, const int64_t* perm, int inverse, hipStream_t s);
hipError_t launch_check_symmetric(const void* y, int dt, int64_t ldy, int64_t n, int64_t* count,
                                 hipStream_t s);
hipError_t launch_hmc_begin(int64_t n, int d, const double* inv_mass, uint64_t seed,
                            const uint64_t* iteration, double* p, int64_t ldp, const double* x,
                            int64_t ldx, const double* grad, const double* loglik, double* x_save,
                            double* g_save, double* l_save, hipStream_t s);
hipError_t launch_hmc_decide(uint64_t seed, uint64_t* iteration, const double* energies,
                             double* flag, double* stats, int64_t* accepted_total, hipStream_t s);
hipError_t launch_hmc_finish(int64_t n, int d, const double* flag, double* x, int64_t ldx,
                             double* grad, double* loglik, const double* x_save,
                             const double* g_save, const double* l_save, hipStream_t s);
hipError_t launch_heldout_count(const void* y, int dt, int64_t ld_y, const uint8_t* missing,
                                int64_t ld_m, const uint8_t* heldout, int64_t ld_h, int64_t n,
                                int64_t* rows, int64_t* total, hipStream_t s);
hipError_t launch_heldout_fill(const void* y, int dt, int64_t ld_y, const uint8_t* missing,
                               int64_t ld_m, const uint8_t* heldout, int64_t ld_h, int64_t n,
                               const int64_t* rows, int64_t capacity, int32_t* pi, int32_t* pj,
                               double* py, hipStream_t s);
hipError_t launch_lpd_accumulate(int64_t m, const int32_t* pi, const int32_t* pj,
                                 const double* py, int d, const double* xs, int64_t ldx,
                                 int64_t xstride, const double* sigmas, int32_t n_draws,
                                 double* acc, int first, hipStream_t s);
hipError_t launch_lpd_finalize(int64_t m, const double* acc, int64_t n_draws, double* part,
                               double* out,
                               hipStream_t s);
hipError_t launch_log_phi(const double* t, double* lnphi, double* mills, int64_t count, int prec,
                          hipStream_t s);
}  // namespace mds

using namespace mds;

namespace {

thread_local char g_last_error[512] = "";
thread_local hipEvent_t g_ev_before = nullptr, g_ev_after = nullptr;

int fail(int status, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return status;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(MDS_ERR_HIP, "%s: %s (%s)", what, hipGetErrorName(e), hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

size_t dtype_size(int dt) { return dt == MDS_F64 ? 8 : 4; }

// Splits a y_dtype argument into the element type (left in y_dtype) and the
// model flags: *truncated = 0 for MDS_UNTRUNCATED.
int split_ytype(int32_t& y_dtype, int* truncated)
{
    const int32_t flags = y_dtype & ~0xFF;
    if (flags & ~MDS_UNTRUNCATED)
        return fail(MDS_ERR_UNSUPPORTED, "unknown model flags 0x%x in y_dtype", (unsigned)flags);
    *truncated = (flags & MDS_UNTRUNCATED) ? 0 : 1;
    y_dtype &= 0xFF;
    return MDS_OK;
}

// Largest LDS a sweep work-group may use (row sums of all its waves).
constexpr size_t kMaxSweepLds = 64 * 1024;

// Tile shape used when the caller passes 0: the autotuner's grid on
// spatially ordered random problems (D = 2, 4, 6; both precisions) rounded
// to one rule per N range, each within a few percent of the grid's best.
// Small problems need short tiles: a wave walks its rows one after another,
// so at N = 1000 8-row tiles (about 1000 one-wave work-groups) fill the chip.
// Up to N ~ 12000 tiles one column group wide whose rows are split over 2 or
// 4 waves keep every wave's walk short, so the last waves of the launch
// finish soon after the others; larger problems run long enough for taller,
// wider tiles, which write fewer partial sums.
void default_tiling(int64_t n, int d, int dtype, int* br, int* wc, int* wr)
{
    (void)dtype;
    if (n <= 1536) {
        *br = 8;
        *wc = 1;
        *wr = 1;
    } else if (n <= 3072) {
        *br = 32;
        *wc = 1;
        *wr = 2;
    } else if (n <= 6144) {
        *br = 64;
        *wc = 1;
        *wr = d <= 2 ? 4 : 2;
    } else if (n <= 12288) {
        *br = 64;
        *wc = 1;
        *wr = 2;
    } else {
        *br = 128;
        *wc = 2;
        *wr = d <= 2 ? 2 : 1;
    }
}

bool pow2_upto8(int v) { return v == 1 || v == 2 || v == 4 || v == 8; }

int resolve_tiling(int64_t n, int d, int dtype, int tile_rows, int tile_waves, Tiling* out)
{
    int br = tile_rows, wc = 0, wr = 1;
    if (tile_waves != 0) {
        if (tile_waves & ~0xFFFF)
            return fail(MDS_ERR_UNSUPPORTED, "tile_waves=0x%x: only bits 0-15 are defined",
                        (unsigned)tile_waves);
        wc = tile_waves & 0xFF;
        wr = (tile_waves >> 8) & 0xFF;
        if (wr == 0) wr = 1;
        if (!pow2_upto8(wc))
            return fail(MDS_ERR_UNSUPPORTED, "tile_waves: %d column waves (must be 1, 2, 4 or 8)",
                        wc);
        if (!pow2_upto8(wr))
            return fail(MDS_ERR_UNSUPPORTED, "tile_waves: %d row waves (must be 1, 2, 4 or 8)",
                        wr);
    }
    if (br == 0 || wc == 0) {
        int dbr, dwc, dwr;
        default_tiling(n, d, dtype, &dbr, &dwc, &dwr);
        if (br == 0) br = dbr;
        if (wc == 0) {
            wc = dwc;
            wr = dwr;
        }
    }
    if (br != 8 && br != 16 && br != 32 && br != 64 && br != 128 && br != 256)
        return fail(MDS_ERR_UNSUPPORTED, "tile_rows=%d: must be 8, 16, 32, 64, 128 or 256", br);
    if (wc * wr > 8)
        return fail(MDS_ERR_UNSUPPORTED, "%d x %d waves per tile: at most 8", wc, wr);
    if (br / wr < 8)
        return fail(MDS_ERR_UNSUPPORTED, "tile_rows=%d split over %d row waves: each needs >= 8 rows",
                    br, wr);
    const int cw = kWave * wc;
    if (!(br % cw == 0 || cw % br == 0))
        return fail(MDS_ERR_UNSUPPORTED, "tile_rows=%d and 64*tile_waves=%d: neither divides the other",
                    br, cw);
    // staged rows hold Y's element type; a model flag in dtype's high bits
    // does not change it
    *out = make_tiling(n, br, wc, wr, (dtype & 0xff) == MDS_F32 ? 4 : 8);
    // one work-group per tile, indexed in 32 bits
    if (out->ntiles > INT32_MAX)
        return fail(MDS_ERR_UNSUPPORTED, "tile %dx%d at n=%lld gives %lld tiles (max 2^31-1)", br,
                    cw, (long long)n, (long long)out->ntiles);
    if (sweep_lds_bytes(*out, d) > kMaxSweepLds)
        return fail(MDS_ERR_UNSUPPORTED, "tile %dx%d with D=%d needs %zu B of LDS (max %zu)", br,
                    cw, d, sweep_lds_bytes(*out, d), kMaxSweepLds);
    return MDS_OK;
}

// the tile_waves value of a resolved tiling (a plain count when wr = 1)
int32_t packed_waves(const Tiling& t) { return t.wr == 1 ? t.wc : (t.wc | (t.wr << 8)); }

int check_problem(int64_t n, int32_t d, const double* x, int64_t ldx, const void* y,
                  int32_t y_dtype, int64_t ldy, const double* sigma_dev)
{
    if (n < 0 || n > MDS_MAX_N) return fail(MDS_ERR_INVALID_ARGUMENT, "n=%lld out of [0, %lld]",
                                            (long long)n, (long long)MDS_MAX_N);
    if (d < 1 || d > MDS_MAX_DIM)
        return fail(MDS_ERR_UNSUPPORTED, "d=%d: supported latent dimensions are 1..%d", d,
                    MDS_MAX_DIM);
    if (y_dtype != MDS_F64 && y_dtype != MDS_F32)
        return fail(MDS_ERR_UNSUPPORTED, "y_dtype=%d: must be MDS_F64 or MDS_F32", y_dtype);
    if (n > 0 && !x) return fail(MDS_ERR_INVALID_ARGUMENT, "x is NULL");
    if (ldx < d) return fail(MDS_ERR_INVALID_ARGUMENT, "ldx=%lld < d=%d", (long long)ldx, d);
    if (n > 1 && !y) return fail(MDS_ERR_INVALID_ARGUMENT, "y is NULL");
    if (n > 0 && ldy < n)
        return fail(MDS_ERR_INVALID_ARGUMENT, "ldy=%lld < n=%lld", (long long)ldy, (long long)n);
    // a wave addresses the rows of its tile (at most 256) by 32-bit byte
    // offsets from its first row; 257 rows of Y must span less than 2^31
    // bytes (ldy below about 10^6 elements: far beyond any Y that fits a GPU)
    if (n > 1 && ldy > (((int64_t)1 << 31) - 1) / (257 * (int64_t)dtype_size(y_dtype)))
        return fail(MDS_ERR_UNSUPPORTED, "ldy=%lld: rows of Y too long for 32-bit offsets",
                    (long long)ldy);
    if (!sigma_dev) return fail(MDS_ERR_INVALID_ARGUMENT, "sigma_dev is NULL");
    if (!aligned(x, 8) || !aligned(sigma_dev, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "x and sigma_dev must be 8-byte aligned");
    if (!aligned(y, dtype_size(y_dtype)))
        return fail(MDS_ERR_INVALID_ARGUMENT, "y is not aligned to its element size");
    return MDS_OK;
}

int check_workspace(const Tiling& t, int d, const void* ws, size_t ws_bytes,
                    WorkspaceLayout* lay)
{
    *lay = workspace_layout(t, d);
    if (ws_bytes < lay->total)
        return fail(MDS_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu B < %zu B needed", ws_bytes,
                    lay->total);
    if (lay->total > 0 && !ws) return fail(MDS_ERR_INVALID_ARGUMENT, "workspace is NULL");
    if (!aligned(ws, MDS_WORKSPACE_ALIGN))
        return fail(MDS_ERR_INVALID_ARGUMENT, "workspace must be %d-byte aligned",
                    MDS_WORKSPACE_ALIGN);
    return MDS_OK;
}

// the arguments of mds_gradient other than its workspace and tiling
int check_gradient_args(int64_t n, int32_t d, const double* x, int64_t ldx, const void* y,
                        int32_t y_dtype, int64_t ldy, const double* sigma_dev,
                        const double* scale_dev, const double* grad, int64_t ldg,
                        const double* loglik_dev, const double* dsigma_dev,
                        const double* dlogsigma_dev)
{
    const int st = check_problem(n, d, x, ldx, y, y_dtype, ldy, sigma_dev);
    if (st) return st;
    if (n > 0 && !grad) return fail(MDS_ERR_INVALID_ARGUMENT, "grad is NULL");
    if (ldg < d) return fail(MDS_ERR_INVALID_ARGUMENT, "ldg=%lld < d=%d", (long long)ldg, d);
    if (!aligned(grad, 8) || !aligned(loglik_dev, 8) || !aligned(dsigma_dev, 8) ||
        !aligned(dlogsigma_dev, 8) || !aligned(scale_dev, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned output pointer");
    return MDS_OK;
}

// a sweep launch, bracketed by the diagnostic events when they are set
hipError_t timed_sweep(int y_dtype, int d, bool grad, const Tiling& t, const SweepArgs& a,
                       hipStream_t s)
{
    return launch_sweep(y_dtype, d, grad, t, a, s, g_ev_before, g_ev_after);
}

// diagnostics: where single-problem sweeps write their per-wave clocks
thread_local unsigned long long* g_tile_trace = nullptr;

SweepArgs sweep_args(const Tiling& t, const WorkspaceLayout& lay, void* ws, int64_t n,
                     const double* x, int64_t ldx, const void* y, int64_t ldy,
                     const double* sigma, int truncated)
{
    char* base = static_cast<char*>(ws);
    SweepArgs a;
    a.n = n;
    a.x = x;
    a.ldx = ldx;
    a.y = y;
    a.ldy = ldy;
    a.sigma = sigma;
    a.truncated = truncated;
    a.br = t.br;
    a.cw = t.cw;
    a.nrb = t.nrb;
    a.wc = t.wc;
    a.wr = t.wr;
    a.rowpart = reinterpret_cast<double*>(base + lay.rowpart);
    a.colpart = reinterpret_cast<double*>(base + lay.colpart);
    a.tscal = reinterpret_cast<double*>(base + lay.tscal);
    a.tcount = reinterpret_cast<uint32_t*>(base + lay.tcount);
    a.trace = g_tile_trace;
    return a;
}

FinalizeArgs finalize_args(const Tiling& t, const SweepArgs& s)
{
    FinalizeArgs f = {};
    f.n = t.n;
    f.br = t.br;
    f.cw = t.cw;
    f.nrb = t.nrb;
    f.ntiles = t.ntiles;
    f.rowpart = s.rowpart;
    f.colpart = s.colpart;
    f.tscal = s.tscal;
    f.tcount = s.tcount;
    f.sigma = s.sigma;
    return f;
}

// Scratch of mds_gradient_noalloc: the partial sums of one evaluation, in a
// static device array (each device holds its own copy for the life of the
// process).  Host code never uses the array's name as an address: its device
// address comes from hipGetSymbolAddress, once per device.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (looked up on the device's first
// call); MDS_OK or MDS_ERR_HIP.
int static_scratch(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(MDS_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr || !aligned(ptr, MDS_WORKSPACE_ALIGN))
            return fail(MDS_ERR_HIP, "static scratch at %p is not %d-byte aligned", ptr,
                        MDS_WORKSPACE_ALIGN);
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MDS_OK;
}

}  // namespace

extern "C" {

const char* mds_status_string(int status)
{
    switch (status) {
        case MDS_OK: return "MDS_OK";
        case MDS_ERR_INVALID_ARGUMENT: return "MDS_ERR_INVALID_ARGUMENT";
        case MDS_ERR_UNSUPPORTED: return "MDS_ERR_UNSUPPORTED";
        case MDS_ERR_WORKSPACE_TOO_SMALL: return "MDS_ERR_WORKSPACE_TOO_SMALL";
        case MDS_ERR_HIP: return "MDS_ERR_HIP";
        case MDS_ERR_NOT_SYMMETRIC: return "MDS_ERR_NOT_SYMMETRIC";
        default: return "MDS_UNKNOWN_STATUS";
    }
}

const char* mds_last_error(void) { return g_last_error; }

int mds_version(void) { return 1 * 10000 + 0 * 100 + 0; }

int mds_workspace_bytes(int64_t n, int32_t d, int32_t y_dtype, int32_t tile_rows,
                        int32_t tile_waves, size_t* bytes)
{
    int trunc = 1;
    {
        const int sst = split_ytype(y_dtype, &trunc);
        if (sst) return sst;
    }
    (void)trunc;
    if (!bytes) return fail(MDS_ERR_INVALID_ARGUMENT, "bytes is NULL");
    if (n < 0 || n > MDS_MAX_N) return fail(MDS_ERR_INVALID_ARGUMENT, "n out of range");
    if (d < 1 || d > MDS_MAX_DIM) return fail(MDS_ERR_UNSUPPORTED, "d=%d unsupported", d);
    if (y_dtype != MDS_F64 && y_dtype != MDS_F32)
        return fail(MDS_ERR_UNSUPPORTED, "y_dtype=%d unsupported", y_dtype);
    Tiling t;
    int st = resolve_tiling(n, d, y_dtype, tile_rows, tile_waves, &t);
    if (st) return st;
    *bytes = workspace_layout(t, d).total;
    return MDS_OK;
}

int mds_resolve_tiling(int64_t n, int32_t d, int32_t y_dtype, int32_t tile_rows,
                       int32_t tile_waves, int32_t* rows_out, int32_t* waves_out)
{
    int trunc = 1;
    {
        const int sst = split_ytype(y_dtype, &trunc);
        if (sst) return sst;
    }
    (void)trunc;
    if (n < 0 || n > MDS_MAX_N) return fail(MDS_ERR_INVALID_ARGUMENT, "n out of range");
    if (d < 1 || d > MDS_MAX_DIM)
        return fail(MDS_ERR_UNSUPPORTED, "d=%d: must be 1..%d", d, MDS_MAX_DIM);
    if (y_dtype != MDS_F64 && y_dtype != MDS_F32)
        return fail(MDS_ERR_UNSUPPORTED, "y_dtype must be MDS_F64 or MDS_F32");
    if (!rows_out || !waves_out) return fail(MDS_ERR_INVALID_ARGUMENT, "output pointer NULL");
    Tiling t;
    const int st = resolve_tiling(n, d, y_dtype, tile_rows, tile_waves, &t);
    if (st) return st;
    *rows_out = t.br;
    *waves_out = packed_waves(t);
    return MDS_OK;
}

int mds_prepare_y(const void* y_src, int32_t src_dtype, int64_t ld_src, const uint8_t* missing,
                  int64_t ld_mask, void* y_out, int32_t out_dtype, int64_t ldy, int64_t n,
                  const int64_t* perm, int64_t* m_obs_dev, hipStream_t stream)
{
    if (n < 0 || n > MDS_MAX_N) return fail(MDS_ERR_INVALID_ARGUMENT, "n out of range");
    if ((src_dtype != MDS_F64 && src_dtype != MDS_F32) ||
        (out_dtype != MDS_F64 && out_dtype != MDS_F32))
        return fail(MDS_ERR_UNSUPPORTED, "dtype must be MDS_F64 or MDS_F32");
    if (n > 0 && (!y_src || !y_out)) return fail(MDS_ERR_INVALID_ARGUMENT, "y_src/y_out NULL");
    if (ld_src < n || ldy < n) return fail(MDS_ERR_INVALID_ARGUMENT, "leading dimension < n");
    if (missing && ld_mask < n) return fail(MDS_ERR_INVALID_ARGUMENT, "ld_mask < n");
    if (!aligned(y_src, dtype_size(src_dtype)) || !aligned(y_out, dtype_size(out_dtype)) ||
        !aligned(m_obs_dev, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    if (y_src == y_out && n > 0 && (src_dtype != out_dtype || ld_src != ldy))
        return fail(MDS_ERR_INVALID_ARGUMENT, "in-place prepare needs equal dtype and stride");
    if (y_src == y_out && n > 0 && perm)
        return fail(MDS_ERR_INVALID_ARGUMENT, "a relabelling prepare cannot run in place");
    if (!aligned(perm, 8)) return fail(MDS_ERR_INVALID_ARGUMENT, "perm misaligned");
    hipError_t e = launch_prepare(y_src, src_dtype, ld_src, missing, ld_mask, y_out, out_dtype,
                                  ldy, n, perm, m_obs_dev, stream);
    if (e != hipSuccess) return hip_fail(e, "prepare launch");
    return MDS_OK;
}

int mds_check_symmetric(const void* y, int32_t y_dtype, int64_t ldy, int64_t n,
                        int64_t* mismatches_dev, hipStream_t stream)
{
    if (n < 0 || n > MDS_MAX_N) return fail(MDS_ERR_INVALID_ARGUMENT, "n out of range");
    if (y_dtype != MDS_F64 && y_dtype != MDS_F32)
        return fail(MDS_ERR_UNSUPPORTED, "y_dtype must be MDS_F64 or MDS_F32");
    if (!mismatches_dev || (n > 0 && !y))
        return fail(MDS_ERR_INVALID_ARGUMENT, "y and mismatches_dev must be non-NULL");
    if (ldy < n) return fail(MDS_ERR_INVALID_ARGUMENT, "ldy < n");
    if (!aligned(y, dtype_size(y_dtype)) || !aligned(mismatches_dev, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    hipError_t e = launch_check_symmetric(y, y_dtype, ldy, n, mismatches_dev, stream);
    if (e != hipSuccess) return hip_fail(e, "symmetry check launch");
    return MDS_OK;
}

int mds_require_symmetric(const void* y, int32_t y_dtype, int64_t ldy, int64_t n,
                          int64_t* mismatches_dev, hipStream_t stream)
{
    const int st = mds_check_symmetric(y, y_dtype, ldy, n, mismatches_dev, stream);
    if (st) return st;
    int64_t bad = 0;
    hipError_t e = hipMemcpyAsync(&bad, mismatches_dev, sizeof(bad), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "symmetry count read-back");
    if (bad)
        return fail(MDS_ERR_NOT_SYMMETRIC, "%lld pairs i > j with y[i][j] != y[j][i] (Y or its "
                    "missing-pair mask is not symmetric)", (long long)bad);
    return MDS_OK;
}

int mds_order_workspace_bytes(int64_t n, size_t* bytes)
{
    if (n < 0 || n > MDS_MAX_N) return fail(MDS_ERR_INVALID_ARGUMENT, "n out of range");
    if (!bytes) return fail(MDS_ERR_INVALID_ARGUMENT, "bytes is NULL");
    *bytes = order_workspace_bytes(n);
    return MDS_OK;
}

int mds_spatial_order(int64_t n, int32_t d, const double* x, int64_t ldx, int64_t* perm,
                      void* workspace, size_t workspace_bytes, hipStream_t stream)
{
    if (n < 0 || n > MDS_MAX_N) return fail(MDS_ERR_INVALID_ARGUMENT, "n out of range");
    if (d < 1 || d > MDS_MAX_DIM)
        return fail(MDS_ERR_UNSUPPORTED, "d=%d: must be 1..%d", d, MDS_MAX_DIM);
    if (ldx < d) return fail(MDS_ERR_INVALID_ARGUMENT, "ldx < d");
    if (n > 0 && (!x || !perm || !workspace))
        return fail(MDS_ERR_INVALID_ARGUMENT, "x, perm and workspace must be non-NULL");
    if (!aligned(x, 8) || !aligned(perm, 8) || !aligned(workspace, MDS_WORKSPACE_ALIGN))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    if (workspace_bytes < order_workspace_bytes(n))
        return fail(MDS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed",
                    workspace_bytes, order_workspace_bytes(n));
    hipError_t e = launch_order(n, d, x, ldx, perm, workspace, stream);
    if (e != hipSuccess) return hip_fail(e, "order launch");
    return MDS_OK;
}

int mds_permute_rows(int64_t n, int32_t d, const double* src, int64_t ld_src, double* dst,
                     int64_t ld_dst, const int64_t* perm, int32_t inverse, hipStream_t stream)
{
    if (n < 0 || n > MDS_MAX_N) return fail(MDS_ERR_INVALID_ARGUMENT, "n out of range");
    if (d < 1 || d > MDS_MAX_DIM)
        return fail(MDS_ERR_UNSUPPORTED, "d=%d: must be 1..%d", d, MDS_MAX_DIM);
    if (ld_src < d || ld_dst < d) return fail(MDS_ERR_INVALID_ARGUMENT, "leading dimension < d");
    if (n > 0 && (!src || !dst || !perm))
        return fail(MDS_ERR_INVALID_ARGUMENT, "src, dst and perm must be non-NULL");
    if (n > 0 && src == dst) return fail(MDS_ERR_INVALID_ARGUMENT, "src and dst must differ");
    if (!aligned(src, 8) || !aligned(dst, 8) || !aligned(perm, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    hipError_t e = launch_permute_rows(n, d, src, ld_src, dst, ld_dst, perm, inverse, stream);
    if (e != hipSuccess) return hip_fail(e, "permute launch");
    return MDS_OK;
}

int mds_loglik(int64_t n, int32_t d, const double* x, int64_t ldx, const void* y,
               int32_t y_dtype, int64_t ldy, const double* sigma_dev, double* loglik_dev,
               void* workspace, size_t workspace_bytes, int32_t tile_rows, int32_t tile_waves,
               hipStream_t stream)
{
    int trunc = 1;
    {
        const int sst = split_ytype(y_dtype, &trunc);
        if (sst) return sst;
    }
    int st = check_problem(n, d, x, ldx, y, y_dtype, ldy, sigma_dev);
    if (st) return st;
    if (!loglik_dev || !aligned(loglik_dev, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "loglik_dev NULL or misaligned");
    Tiling t;
    if ((st = resolve_tiling(n, d, y_dtype, tile_rows, tile_waves, &t))) return st;
    WorkspaceLayout lay;
    if ((st = check_workspace(t, d, workspace, workspace_bytes, &lay))) return st;

    SweepArgs sa = sweep_args(t, lay, workspace, n, x, ldx, y, ldy, sigma_dev, trunc);
    hipError_t e = timed_sweep(y_dtype, d, false, t, sa, stream);
    if (e != hipSuccess) return hip_fail(e, "sweep launch");
    FinalizeArgs fa = finalize_args(t, sa);
    fa.loglik = loglik_dev;
    e = launch_finalize(d, fa, stream);
    if (e != hipSuccess) return hip_fail(e, "finalize launch");
    return MDS_OK;
}

int mds_gradient(int64_t n, int32_t d, const double* x, int64_t ldx, const void* y,
                 int32_t y_dtype, int64_t ldy, const double* sigma_dev, const double* scale_dev,
                 double* grad, int64_t ldg, double* loglik_dev, double* dsigma_dev,
                 double* dlogsigma_dev, void* workspace, size_t workspace_bytes,
                 int32_t tile_rows, int32_t tile_waves, hipStream_t stream)
{
    int trunc = 1;
    {
        const int sst = split_ytype(y_dtype, &trunc);
        if (sst) return sst;
    }
    int st = check_gradient_args(n, d, x, ldx, y, y_dtype, ldy, sigma_dev, scale_dev, grad, ldg,
                                 loglik_dev, dsigma_dev, dlogsigma_dev);
    if (st) return st;
    Tiling t;
    if ((st = resolve_tiling(n, d, y_dtype, tile_rows, tile_waves, &t))) return st;
    WorkspaceLayout lay;
    if ((st = check_workspace(t, d, workspace, workspace_bytes, &lay))) return st;

    SweepArgs sa = sweep_args(t, lay, workspace, n, x, ldx, y, ldy, sigma_dev, trunc);
    hipError_t e = timed_sweep(y_dtype, d, true, t, sa, stream);
    if (e != hipSuccess) return hip_fail(e, "sweep launch");
    FinalizeArgs fa = finalize_args(t, sa);
    fa.scale = scale_dev;
    fa.grad = grad;
    fa.ldg = ldg;
    fa.loglik = loglik_dev;
    fa.dsigma = dsigma_dev;
    fa.dlogsigma = dlogsigma_dev;
    e = launch_finalize(d, fa, stream);
    if (e != hipSuccess) return hip_fail(e, "finalize launch");
    return MDS_OK;
}

size_t mds_noalloc_scratch_bytes(void) { return kStaticScratchBytes; }

int mds_gradient_noalloc(int64_t n, int32_t d, const double* x, int64_t ldx, const void* y,
                         int32_t y_dtype, int64_t ldy, const double* sigma_dev,
                         const double* scale_dev, double* grad, int64_t ldg, double* loglik_dev,
                         double* dsigma_dev, double* dlogsigma_dev, int32_t tile_rows,
                         int32_t tile_waves, hipStream_t stream)
{
    // every argument is validated before the scratch lookup (a HIP call)
    int st = 0;
    {
        int32_t yt = y_dtype;
        int trunc = 1;
        if ((st = split_ytype(yt, &trunc))) return st;
        st = check_gradient_args(n, d, x, ldx, y, yt, ldy, sigma_dev, scale_dev, grad, ldg,
                                 loglik_dev, dsigma_dev, dlogsigma_dev);
        if (st) return st;
    }
    // the workspace this evaluation needs must fit the static scratch
    size_t need = 0;
    if ((st = mds_workspace_bytes(n, d, y_dtype, tile_rows, tile_waves, &need))) return st;
    if (need > kStaticScratchBytes)
        return fail(MDS_ERR_WORKSPACE_TOO_SMALL,
                    "n=%lld d=%d needs %zu B of partial sums; the static scratch of "
                    "mds_gradient_noalloc holds %zu B (use mds_gradient with a workspace)",
                    (long long)n, d, need, kStaticScratchBytes);
    void* ws = nullptr;
    if ((st = static_scratch(&ws))) return st;
    // every slot of the partial sums that the finalize reads is written by the
    // sweep of the same call, so nothing needs clearing between calls
    return mds_gradient(n, d, x, ldx, y, y_dtype, ldy, sigma_dev, scale_dev, grad, ldg,
                        loglik_dev, dsigma_dev, dlogsigma_dev, ws, kStaticScratchBytes,
                        tile_rows, tile_waves, stream);
}

int mds_leapfrog(int64_t n, int32_t d, double* x, int64_t ldx, double* p, int64_t ldp,
                 const void* y, int32_t y_dtype, int64_t ldy, const double* sigma_dev,
                 const double* inv_mass, const double* step_dev, const double* prior_dev,
                 int32_t n_steps, double* grad_io, double* loglik_io, int32_t cache_valid,
                 double* energy_start_dev, double* energy_end_dev, void* workspace,
                 size_t workspace_bytes, int32_t tile_rows, int32_t tile_waves,
                 hipStream_t stream)
{
    int trunc = 1;
    {
        const int sst = split_ytype(y_dtype, &trunc);
        if (sst) return sst;
    }
    int st = check_problem(n, d, x, ldx, y, y_dtype, ldy, sigma_dev);
    if (st) return st;
    if (n > 0 && (!p || !grad_io)) return fail(MDS_ERR_INVALID_ARGUMENT, "p or grad_io is NULL");
    if (ldp < d) return fail(MDS_ERR_INVALID_ARGUMENT, "ldp=%lld < d=%d", (long long)ldp, d);
    if (!loglik_io || !step_dev) return fail(MDS_ERR_INVALID_ARGUMENT, "loglik_io or step_dev NULL");
    if (n_steps < 0) return fail(MDS_ERR_INVALID_ARGUMENT, "n_steps=%d < 0", n_steps);
    if (!aligned(p, 8) || !aligned(grad_io, 8) || !aligned(loglik_io, 8) ||
        !aligned(step_dev, 8) || !aligned(prior_dev, 8) || !aligned(inv_mass, 8) ||
        !aligned(energy_start_dev, 8) || !aligned(energy_end_dev, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    if (n > 0 && (x == p || x == grad_io || p == grad_io))
        return fail(MDS_ERR_INVALID_ARGUMENT, "x, p and grad_io must not alias");
    Tiling t;
    if ((st = resolve_tiling(n, d, y_dtype, tile_rows, tile_waves, &t))) return st;
    WorkspaceLayout lay;
    if ((st = check_workspace(t, d, workspace, workspace_bytes, &lay))) return st;

    SweepArgs sa = sweep_args(t, lay, workspace, n, x, ldx, y, ldy, sigma_dev, trunc);
    hipError_t e;

    // grad log pi and L at a point: sweep + finalize, optionally followed by
    // a kick of mult*eps and a drift of eps, fused into the finalize
    auto evaluate = [&](double mult, int kick, int drift) -> int {
        hipError_t err = timed_sweep(y_dtype, d, true, t, sa, stream);
        if (err != hipSuccess) return hip_fail(err, "sweep launch");
        FinalizeArgs fa = finalize_args(t, sa);
        fa.grad = grad_io;
        fa.ldg = d;
        fa.loglik = loglik_io;
        fa.prior = prior_dev;
        fa.x = x;
        fa.ldx = ldx;
        fa.p = kick ? p : nullptr;
        fa.ldp = ldp;
        fa.inv_mass = inv_mass;
        fa.step = step_dev;
        fa.kick_mult = mult;
        fa.drift = drift;
        err = launch_finalize(d, fa, stream);
        if (err != hipSuccess) return hip_fail(err, "finalize launch");
        return MDS_OK;
    };

    // first half kick (fused into the first evaluation when possible)
    const bool fuse_first = !cache_valid && !energy_start_dev && n_steps > 0;
    if (!cache_valid) {
        if ((st = evaluate(0.5, fuse_first ? 1 : 0, fuse_first ? 1 : 0))) return st;
    }
    if (energy_start_dev) {
        e = launch_energy(n, d, x, ldx, p, ldp, inv_mass, prior_dev, loglik_io, energy_start_dev,
                          stream);
        if (e != hipSuccess) return hip_fail(e, "energy launch");
    }
    if (n_steps > 0 && !fuse_first) {
        e = launch_kick_drift(n, d, x, ldx, p, ldp, grad_io, inv_mass, step_dev, 0.5, 1, stream);
        if (e != hipSuccess) return hip_fail(e, "kick launch");
    }
    for (int s = 1; s <= n_steps; ++s) {
        const bool last = (s == n_steps);
        if ((st = evaluate(last ? 0.5 : 1.0, 1, last ? 0 : 1))) return st;
    }
    if (energy_end_dev) {
        e = launch_energy(n, d, x, ldx, p, ldp, inv_mass, prior_dev, loglik_io, energy_end_dev,
                          stream);
        if (e != hipSuccess) return hip_fail(e, "energy launch");
    }
    return MDS_OK;
}

// HMC workspace: the gradient workspace, then the saved x and gradient
// (n*d doubles each) and four scalars (saved L, H_start, H_end, decision)
struct HmcLayout {
    size_t x_save, g_save, scal, total;
};

static HmcLayout hmc_layout(const WorkspaceLayout& lay, int64_t n, int d)
{
    HmcLayout h;
    const size_t nd = (size_t)n * d * sizeof(double);
    h.x_save = align_up(lay.total, 256);
    h.g_save = align_up(h.x_save + nd, 256);
    h.scal = align_up(h.g_save + nd, 256);
    h.total = align_up(h.scal + 4 * sizeof(double), 256);
    return h;
}

int mds_hmc_workspace_bytes(int64_t n, int32_t d, int32_t y_dtype, int32_t tile_rows,
                            int32_t tile_waves, size_t* bytes)
{
    int trunc = 1;
    {
        const int sst = split_ytype(y_dtype, &trunc);
        if (sst) return sst;
    }
    (void)trunc;
    if (!bytes) return fail(MDS_ERR_INVALID_ARGUMENT, "bytes is NULL");
    if (n < 0 || n > MDS_MAX_N) return fail(MDS_ERR_INVALID_ARGUMENT, "n out of range");
    if (d < 1 || d > MDS_MAX_DIM)
        return fail(MDS_ERR_UNSUPPORTED, "d=%d: must be 1..%d", d, MDS_MAX_DIM);
    if (y_dtype != MDS_F64 && y_dtype != MDS_F32)
        return fail(MDS_ERR_UNSUPPORTED, "y_dtype must be MDS_F64 or MDS_F32");
    Tiling t;
    const int st = resolve_tiling(n, d, y_dtype, tile_rows, tile_waves, &t);
    if (st) return st;
    *bytes = hmc_layout(workspace_layout(t, d), n, d).total;
    return MDS_OK;
}

int mds_hmc_momentum(int64_t n, int32_t d, const double* inv_mass, uint64_t seed,
                     const uint64_t* iteration_dev, double* p, int64_t ldp, hipStream_t stream)
{
    if (n < 0 || n > MDS_MAX_N) return fail(MDS_ERR_INVALID_ARGUMENT, "n out of range");
    if (d < 1 || d > MDS_MAX_DIM)
        return fail(MDS_ERR_UNSUPPORTED, "d=%d: must be 1..%d", d, MDS_MAX_DIM);
    if (!iteration_dev || (n > 0 && !p))
        return fail(MDS_ERR_INVALID_ARGUMENT, "iteration_dev and p must be non-NULL");
    if (ldp < d) return fail(MDS_ERR_INVALID_ARGUMENT, "ldp < d");
    if (!aligned(iteration_dev, 8) || !aligned(p, 8) || !aligned(inv_mass, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    hipError_t e = launch_hmc_begin(n, d, inv_mass, seed, iteration_dev, p, ldp, nullptr, 0,
                                    nullptr, nullptr, nullptr, nullptr, nullptr, stream);
    if (e != hipSuccess) return hip_fail(e, "momentum launch");
    return MDS_OK;
}

int mds_hmc_step(int64_t n, int32_t d, double* x, int64_t ldx, const void* y, int32_t y_dtype,
                 int64_t ldy, const double* sigma_dev, const double* inv_mass,
                 const double* step_dev, const double* prior_dev, int32_t n_steps,
                 uint64_t seed, uint64_t* iteration_dev, double* p, int64_t ldp,
                 double* grad_io, double* loglik_io, int32_t cache_valid, double* stats_dev,
                 int64_t* accepted_total_dev, void* workspace, size_t workspace_bytes,
                 int32_t tile_rows, int32_t tile_waves, hipStream_t stream)
{
    const int32_t y_arg = y_dtype;  // with its model flags, for the leapfrog calls
    int trunc = 1;
    {
        const int sst = split_ytype(y_dtype, &trunc);
        if (sst) return sst;
    }
    (void)trunc;
    int st = check_problem(n, d, x, ldx, y, y_dtype, ldy, sigma_dev);
    if (st) return st;
    if (!iteration_dev || !aligned(iteration_dev, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "iteration_dev NULL or misaligned");
    if (!aligned(stats_dev, 8) || !aligned(accepted_total_dev, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    Tiling t;
    if ((st = resolve_tiling(n, d, y_dtype, tile_rows, tile_waves, &t))) return st;
    const WorkspaceLayout lay = workspace_layout(t, d);
    const HmcLayout h = hmc_layout(lay, n, d);
    if (!workspace || !aligned(workspace, MDS_WORKSPACE_ALIGN))
        return fail(MDS_ERR_INVALID_ARGUMENT, "workspace NULL or not %d-byte aligned",
                    MDS_WORKSPACE_ALIGN);
    if (workspace_bytes < h.total)
        return fail(MDS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed",
                    workspace_bytes, h.total);
    char* base = static_cast<char*>(workspace);
    double* x_save = reinterpret_cast<double*>(base + h.x_save);
    double* g_save = reinterpret_cast<double*>(base + h.g_save);
    double* scal = reinterpret_cast<double*>(base + h.scal);  // L_save, H0, H1, decision

    // grad log pi and L at x, when the caller has no cached values
    if (!cache_valid) {
        st = mds_leapfrog(n, d, x, ldx, p, ldp, y, y_arg, ldy, sigma_dev, inv_mass, step_dev,
                          prior_dev, 0, grad_io, loglik_io, 0, nullptr, nullptr, workspace,
                          lay.total, tile_rows, tile_waves, stream);
        if (st) return st;
    }
    hipError_t e = launch_hmc_begin(n, d, inv_mass, seed, iteration_dev, p, ldp, x, ldx, grad_io,
                                    loglik_io, x_save, g_save, scal, stream);
    if (e != hipSuccess) return hip_fail(e, "momentum launch");
    st = mds_leapfrog(n, d, x, ldx, p, ldp, y, y_arg, ldy, sigma_dev, inv_mass, step_dev,
                      prior_dev, n_steps, grad_io, loglik_io, 1, scal + 1, scal + 2, workspace,
                      lay.total, tile_rows, tile_waves, stream);
    if (st) return st;
    e = launch_hmc_decide(seed, iteration_dev, scal + 1, scal + 3, stats_dev, accepted_total_dev,
                          stream);
    if (e != hipSuccess) return hip_fail(e, "decision launch");
    e = launch_hmc_finish(n, d, scal + 3, x, ldx, grad_io, loglik_io, x_save, g_save, scal,
                          stream);
    if (e != hipSuccess) return hip_fail(e, "restore launch");
    return MDS_OK;
}

int mds_heldout_workspace_bytes(int64_t n, size_t* bytes)
{
    if (!bytes) return fail(MDS_ERR_INVALID_ARGUMENT, "bytes is NULL");
    if (n < 0 || n > MDS_MAX_N) return fail(MDS_ERR_INVALID_ARGUMENT, "n out of range");
    *bytes = align_up((size_t)(n + 1) * sizeof(int64_t), 256);
    return MDS_OK;
}

static int check_heldout_args(const void* y_src, int32_t src_dtype, int64_t ld_src,
                              const uint8_t* missing, int64_t ld_mask, const uint8_t* heldout,
                              int64_t ld_heldout, int64_t n, void* ws, size_t ws_bytes)
{
    if (n < 0 || n > MDS_MAX_N) return fail(MDS_ERR_INVALID_ARGUMENT, "n out of range");
    if (src_dtype != MDS_F64 && src_dtype != MDS_F32)
        return fail(MDS_ERR_UNSUPPORTED, "src_dtype must be MDS_F64 or MDS_F32");
    if (n > 0 && (!y_src || !heldout || !ws))
        return fail(MDS_ERR_INVALID_ARGUMENT, "y_src, heldout and workspace must be non-NULL");
    if (ld_src < n || ld_heldout < n || (missing && ld_mask < n))
        return fail(MDS_ERR_INVALID_ARGUMENT, "leading dimension < n");
    if (!aligned(y_src, dtype_size(src_dtype)) || !aligned(ws, MDS_WORKSPACE_ALIGN))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    size_t need = 0;
    mds_heldout_workspace_bytes(n, &need);
    if (ws_bytes < need)
        return fail(MDS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed", ws_bytes,
                    need);
    return MDS_OK;
}

int mds_heldout_count(const void* y_src, int32_t src_dtype, int64_t ld_src,
                      const uint8_t* missing, int64_t ld_mask, const uint8_t* heldout,
                      int64_t ld_heldout, int64_t n, int64_t* m_dev, void* workspace,
                      size_t workspace_bytes, hipStream_t stream)
{
    int st = check_heldout_args(y_src, src_dtype, ld_src, missing, ld_mask, heldout, ld_heldout,
                                n, workspace, workspace_bytes);
    if (st) return st;
    if (!m_dev || !aligned(m_dev, 8)) return fail(MDS_ERR_INVALID_ARGUMENT, "m_dev NULL or misaligned");
    hipError_t e = launch_heldout_count(y_src, src_dtype, ld_src, missing, ld_mask, heldout,
                                        ld_heldout, n, static_cast<int64_t*>(workspace), m_dev,
                                        stream);
    if (e != hipSuccess) return hip_fail(e, "held-out count launch");
    return MDS_OK;
}

int mds_heldout_fill(const void* y_src, int32_t src_dtype, int64_t ld_src,
                     const uint8_t* missing, int64_t ld_mask, const uint8_t* heldout,
                     int64_t ld_heldout, int64_t n, const void* workspace, size_t workspace_bytes,
                     int64_t capacity, int32_t* pi, int32_t* pj, double* py, hipStream_t stream)
{
    int st = check_heldout_args(y_src, src_dtype, ld_src, missing, ld_mask, heldout, ld_heldout,
                                n, const_cast<void*>(workspace), workspace_bytes);
    if (st) return st;
    if (capacity < 0) return fail(MDS_ERR_INVALID_ARGUMENT, "capacity < 0");
    if (capacity > 0 && (!pi || !pj || !py))
        return fail(MDS_ERR_INVALID_ARGUMENT, "pair arrays must be non-NULL");
    if (!aligned(pi, 4) || !aligned(pj, 4) || !aligned(py, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    hipError_t e = launch_heldout_fill(y_src, src_dtype, ld_src, missing, ld_mask, heldout,
                                       ld_heldout, n, static_cast<const int64_t*>(workspace),
                                       capacity, pi, pj, py, stream);
    if (e != hipSuccess) return hip_fail(e, "held-out fill launch");
    return MDS_OK;
}

int mds_lpd_accumulate(int64_t m, const int32_t* pi, const int32_t* pj, const double* py,
                       int32_t d, const double* x, int64_t ldx, const double* sigma_dev,
                       double* acc, int32_t first, hipStream_t stream)
{
    if (m < 0) return fail(MDS_ERR_INVALID_ARGUMENT, "m < 0");
    if (d < 1 || d > MDS_MAX_DIM)
        return fail(MDS_ERR_UNSUPPORTED, "d=%d: must be 1..%d", d, MDS_MAX_DIM);
    if (ldx < d) return fail(MDS_ERR_INVALID_ARGUMENT, "ldx < d");
    if (m > 0 && (!pi || !pj || !py || !x || !sigma_dev || !acc))
        return fail(MDS_ERR_INVALID_ARGUMENT, "NULL pointer");
    if (!aligned(pi, 4) || !aligned(pj, 4) || !aligned(py, 8) || !aligned(x, 8) ||
        !aligned(sigma_dev, 8) || !aligned(acc, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    hipError_t e = launch_lpd_accumulate(m, pi, pj, py, d, x, ldx, 0, sigma_dev, 1, acc,
                                         first ? 1 : 0, stream);
    if (e != hipSuccess) return hip_fail(e, "lpd accumulate launch");
    return MDS_OK;
}

int mds_lpd_accumulate_draws(int64_t m, const int32_t* pi, const int32_t* pj, const double* py,
                             int32_t d, const double* xs, int64_t ldx, int64_t draw_stride,
                             const double* sigmas_dev, int32_t n_draws, double* acc,
                             int32_t first, hipStream_t stream)
{
    if (m < 0) return fail(MDS_ERR_INVALID_ARGUMENT, "m < 0");
    if (n_draws < 0) return fail(MDS_ERR_INVALID_ARGUMENT, "n_draws < 0");
    if (d < 1 || d > MDS_MAX_DIM)
        return fail(MDS_ERR_UNSUPPORTED, "d=%d: must be 1..%d", d, MDS_MAX_DIM);
    if (ldx < d) return fail(MDS_ERR_INVALID_ARGUMENT, "ldx < d");
    if (draw_stride < 0) return fail(MDS_ERR_INVALID_ARGUMENT, "draw_stride < 0");
    if (m > 0 && n_draws > 0 && (!pi || !pj || !py || !xs || !sigmas_dev || !acc))
        return fail(MDS_ERR_INVALID_ARGUMENT, "NULL pointer");
    if (!aligned(pi, 4) || !aligned(pj, 4) || !aligned(py, 8) || !aligned(xs, 8) ||
        !aligned(sigmas_dev, 8) || !aligned(acc, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    hipError_t e = launch_lpd_accumulate(m, pi, pj, py, d, xs, ldx, draw_stride, sigmas_dev,
                                         n_draws, acc, first ? 1 : 0, stream);
    if (e != hipSuccess) return hip_fail(e, "lpd accumulate launch");
    return MDS_OK;
}

int mds_lpd_workspace_bytes(int64_t m, size_t* bytes)
{
    if (!bytes) return fail(MDS_ERR_INVALID_ARGUMENT, "bytes is NULL");
    if (m < 0) return fail(MDS_ERR_INVALID_ARGUMENT, "m < 0");
    *bytes = align_up((size_t)kLpdMaxParts * sizeof(double), 256);
    return MDS_OK;
}

int mds_lpd_finalize(int64_t m, const double* acc, int64_t n_draws, void* workspace,
                     size_t workspace_bytes, double* lpd_dev, hipStream_t stream)
{
    if (m < 0 || n_draws < 1) return fail(MDS_ERR_INVALID_ARGUMENT, "m < 0 or n_draws < 1");
    if ((m > 0 && !acc) || !lpd_dev || !workspace)
        return fail(MDS_ERR_INVALID_ARGUMENT, "NULL pointer");
    if (!aligned(acc, 8) || !aligned(lpd_dev, 8) || !aligned(workspace, MDS_WORKSPACE_ALIGN))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    size_t need = 0;
    mds_lpd_workspace_bytes(m, &need);
    if (workspace_bytes < need)
        return fail(MDS_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu needed",
                    workspace_bytes, need);
    hipError_t e = launch_lpd_finalize(m, acc, n_draws, static_cast<double*>(workspace), lpd_dev,
                                       stream);
    if (e != hipSuccess) return hip_fail(e, "lpd finalize launch");
    return MDS_OK;
}

int mds_log_phi(const double* t, double* lnphi, double* mills, int64_t count, int32_t precision,
                hipStream_t stream)
{
    if (count < 0) return fail(MDS_ERR_INVALID_ARGUMENT, "count < 0");
    if (count > 0 && !t) return fail(MDS_ERR_INVALID_ARGUMENT, "t is NULL");
    if (precision != MDS_F64 && precision != MDS_F32)
        return fail(MDS_ERR_UNSUPPORTED, "precision=%d unsupported", precision);
    if (!aligned(t, 8) || !aligned(lnphi, 8) || !aligned(mills, 8))
        return fail(MDS_ERR_INVALID_ARGUMENT, "misaligned pointer");
    hipError_t e = launch_log_phi(t, lnphi, mills, count, precision, stream);
    if (e != hipSuccess) return hip_fail(e, "log_phi launch");
    return MDS_OK;
}

// ---------------------------------------------------------------- batches

namespace {

constexpr int kFinElemsPerBlock = 64;  // finalize element block (one wave wide)

// finalize element blocks of one problem of a batch (none without a gradient)
int64_t batch_elem_blocks(const mds_problem_desc& q)
{
    return q.grad ? (q.n * q.d + kFinElemsPerBlock - 1) / kFinElemsPerBlock : 0;
}
constexpr int32_t kBatchLeapfrogReady = 1;  // mds_batch_plan.flags bit 0
// rows per tile of a batched problem whose descriptor says 0, and the
// batch's waves when tile_waves is 0: 128-row tiles two column groups wide
// (on 64 problems of N ~ U[500, 8000], D in {2, 4, 6}, timed against every
// common wave layout by the batch autotuner: 1.9 ms per evaluation against
// 2.1 ms with four column groups)
constexpr int kBatchDefaultRows = 128;
constexpr int kBatchDefaultWaves = 2;

struct BatchLayout {
    size_t table;   // BatchProblem[count]
    size_t cursor;  // uint64 tile cursor
    size_t blkmap;  // int32[blocks]: the problem of each finalize element block
    int64_t blocks;
    std::vector<size_t> ws;  // per-problem partial buffers
    std::vector<Tiling> tilings;
    size_t total;
};

static int batch_layout(const mds_problem_desc* descs, int32_t count, int32_t y_dtype,
                 int32_t tile_waves, BatchLayout* L, size_t* max_lds)
{
    if (count < 1) return fail(MDS_ERR_INVALID_ARGUMENT, "count=%d < 1", count);
    if (!descs) return fail(MDS_ERR_INVALID_ARGUMENT, "descs is NULL");
    if (y_dtype != MDS_F64 && y_dtype != MDS_F32)
        return fail(MDS_ERR_UNSUPPORTED, "y_dtype=%d unsupported", y_dtype);
    const int waves = tile_waves ? tile_waves : kBatchDefaultWaves;  // packed: column and row waves
    size_t off = 0;
    L->table = off;
    off = align_up(off + sizeof(BatchProblem) * (size_t)count, 256);
    L->cursor = off;
    off = align_up(off + sizeof(unsigned long long), 256);
    // element blocks of the problems that want a gradient
    L->blocks = 0;
    for (int32_t k = 0; k < count; ++k) L->blocks += batch_elem_blocks(descs[k]);
    L->blkmap = off;
    off = align_up(off + sizeof(int32_t) * (size_t)L->blocks, 256);
    L->ws.resize(count);
    L->tilings.resize(count);
    *max_lds = 0;
    for (int32_t k = 0; k < count; ++k) {
        const mds_problem_desc& q = descs[k];
        int st = check_problem(q.n, q.d, q.x, q.ldx, q.y, y_dtype, q.ldy, q.sigma);
        if (st) return fail(st, "problem %d: %s", k, std::string(g_last_error).c_str());
        if (q.grad && q.ldg < q.d) return fail(MDS_ERR_INVALID_ARGUMENT, "problem %d: ldg < d", k);
        if (!aligned(q.grad, 8) || !aligned(q.loglik, 8) || !aligned(q.dsigma, 8) ||
            !aligned(q.dlogsigma, 8) || !aligned(q.scale, 8) || !aligned(q.p, 8) ||
            !aligned(q.step, 8))
            return fail(MDS_ERR_INVALID_ARGUMENT, "problem %d: misaligned pointer", k);
        if (q.p && q.ldp < q.d) return fail(MDS_ERR_INVALID_ARGUMENT, "problem %d: ldp < d", k);
        if (q.n > 0 && q.p && (q.p == q.x || q.p == q.grad || q.x == q.grad))
            return fail(MDS_ERR_INVALID_ARGUMENT, "problem %d: x, p and grad must not alias", k);
        Tiling t;
        if (q.tile_rows == 0 &&
            resolve_tiling(q.n, q.d, y_dtype, kBatchDefaultRows, waves, &t) == MDS_OK) {
            // the batch default: the many problems supply the parallelism, and
            // taller tiles write fewer partial sums
        } else if ((st = resolve_tiling(q.n, q.d, y_dtype, q.tile_rows, waves, &t))) {
            return fail(st, "problem %d: %s", k, std::string(g_last_error).c_str());
        }
        L->tilings[k] = t;
        L->ws[k] = off;
        off = align_up(off + workspace_layout(t, q.d).total, 256);
        const size_t lds = sweep_lds_bytes(t, q.d);
        if (lds > *max_lds) *max_lds = lds;
    }
    L->total = off;
    return MDS_OK;
}

// the block map of an initialised batch: after the table and the cursor
// (the layout of batch_layout)
static const int32_t* batch_blkmap(const mds_batch_plan* plan)
{
    const size_t off = align_up(align_up(sizeof(BatchProblem) * (size_t)plan->count, 256) +
                                    sizeof(unsigned long long), 256);
    return reinterpret_cast<const int32_t*>(static_cast<const char*>(plan->workspace) + off);
}

static int device_cu_count(int* cus)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    return MDS_OK;
}

}  // namespace

int mds_batch_workspace_bytes(const mds_problem_desc* descs, int32_t count, int32_t y_dtype,
                              int32_t tile_waves, size_t* bytes)
{
    if (!bytes) return fail(MDS_ERR_INVALID_ARGUMENT, "bytes is NULL");
    int trunc = 1;
    {
        const int sst = split_ytype(y_dtype, &trunc);
        if (sst) return sst;
    }
    (void)trunc;
    BatchLayout L;
    size_t lds;
    int st = batch_layout(descs, count, y_dtype, tile_waves, &L, &lds);
    if (st) return st;
    *bytes = L.total;
    return MDS_OK;
}

int mds_batch_init(const mds_problem_desc* descs, int32_t count, int32_t y_dtype,
                   int32_t tile_waves, void* workspace, size_t workspace_bytes,
                   mds_batch_plan* plan, hipStream_t stream)
{
    if (!plan) return fail(MDS_ERR_INVALID_ARGUMENT, "plan is NULL");
    int trunc = 1;
    {
        const int sst = split_ytype(y_dtype, &trunc);
        if (sst) return sst;
    }
    BatchLayout L;
    size_t max_lds;
    int st = batch_layout(descs, count, y_dtype, tile_waves, &L, &max_lds);
    if (st) return st;
    if (!workspace) return fail(MDS_ERR_INVALID_ARGUMENT, "workspace is NULL");
    if (!aligned(workspace, MDS_WORKSPACE_ALIGN))
        return fail(MDS_ERR_INVALID_ARGUMENT, "workspace must be %d-byte aligned",
                    MDS_WORKSPACE_ALIGN);
    if (workspace_bytes < L.total)
        return fail(MDS_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu B < %zu B needed",
                    workspace_bytes, L.total);
    // waves per work-group (column x row waves, common to the batch)
    const int waves = L.tilings[0].waves;

    // host image of [table | cursor | block map]; copied in one transfer
    std::vector<unsigned char> img(L.blkmap + sizeof(int32_t) * (size_t)L.blocks, 0);
    BatchProblem* tab = reinterpret_cast<BatchProblem*>(img.data());
    int32_t* blkmap = reinterpret_cast<int32_t*>(img.data() + L.blkmap);
    char* base = static_cast<char*>(workspace);
    int64_t tiles = 0, blocks = 0;
    int leapfrog_ready = 1;
    for (int32_t k = 0; k < count; ++k) {
        const mds_problem_desc& q = descs[k];
        const Tiling& t = L.tilings[k];
        BatchProblem P = {};
        P.sweep = sweep_args(t, workspace_layout(t, q.d), base + L.ws[k], q.n, q.x, q.ldx, q.y,
                             q.ldy, q.sigma, trunc);
        P.sweep.trace = nullptr;  // the per-wave timeline is for single-problem sweeps
        P.d = q.d;
        P.tile_base = tiles;
        P.ntiles = t.ntiles;
        P.blk_base = blocks;
        P.nblk = batch_elem_blocks(q);
        P.scale = q.scale;
        P.grad = q.grad;
        P.ldg = q.ldg;
        P.loglik = q.loglik;
        P.dsigma = q.dsigma;
        P.dlogsigma = q.dlogsigma;
        P.x = const_cast<double*>(q.x);
        P.p = q.p;
        P.ldp = q.ldp;
        P.step = q.step;
        tab[k] = P;
        if (!q.step || !q.loglik || (q.n > 0 && (!q.p || !q.grad))) leapfrog_ready = 0;
        for (int64_t b = 0; b < P.nblk; ++b) blkmap[blocks + b] = k;
        tiles += t.ntiles;
        blocks += P.nblk;
    }
    hipError_t e = hipMemcpyAsync(workspace, img.data(), img.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "batch table upload");

    int cus = 0;
    if ((st = device_cu_count(&cus))) return st;
    int max_d = 1;
    for (int32_t k = 0; k < count; ++k) max_d = descs[k].d > max_d ? descs[k].d : max_d;
    const int per_cu = batch_sweep_blocks_per_cu(y_dtype, true, max_d, waves, max_lds);
    plan->count = count;
    plan->max_d = max_d;
    plan->flags = leapfrog_ready ? kBatchLeapfrogReady : 0;
    plan->y_dtype = y_dtype;
    plan->tile_waves = waves;
    plan->grid = cus * per_cu;
    plan->total_tiles = tiles;
    plan->elem_blocks = blocks;
    plan->lds_bytes = max_lds;
    plan->workspace = workspace;
    plan->workspace_bytes = workspace_bytes;
    return MDS_OK;
}

int mds_batch_eval(const mds_batch_plan* plan, int32_t want_grad, hipStream_t stream)
{
    if (!plan || !plan->workspace || plan->count < 1)
        return fail(MDS_ERR_INVALID_ARGUMENT, "plan is not initialised");
    char* base = static_cast<char*>(plan->workspace);
    const BatchProblem* probs = reinterpret_cast<const BatchProblem*>(base);
    unsigned long long* cursor = reinterpret_cast<unsigned long long*>(
        base + align_up(sizeof(BatchProblem) * (size_t)plan->count, 256));
    hipError_t e = hipSuccess;
    if (g_ev_before && (e = hipEventRecord(g_ev_before, stream)) != hipSuccess)
        return hip_fail(e, "event record");
    e = launch_batch_sweep(plan->y_dtype, want_grad != 0, plan->max_d, probs, plan->count,
                           plan->total_tiles, cursor, plan->tile_waves, plan->lds_bytes,
                           plan->grid, stream);
    if (e != hipSuccess) return hip_fail(e, "batch sweep launch");
    if (g_ev_after && (e = hipEventRecord(g_ev_after, stream)) != hipSuccess)
        return hip_fail(e, "event record");
    e = launch_batch_finalize(probs, batch_blkmap(plan), plan->count,
                              want_grad ? plan->elem_blocks : 0, cursor, 0.0, 0, 0, stream);
    if (e != hipSuccess) return hip_fail(e, "batch finalize launch");
    return MDS_OK;
}

int mds_batch_leapfrog(const mds_batch_plan* plan, int32_t n_steps, int32_t cache_valid,
                       hipStream_t stream)
{
    if (!plan || !plan->workspace || plan->count < 1)
        return fail(MDS_ERR_INVALID_ARGUMENT, "plan is not initialised");
    if (!(plan->flags & kBatchLeapfrogReady))
        return fail(MDS_ERR_INVALID_ARGUMENT,
                    "every problem needs p, step, grad and loglik for the leapfrog");
    if (n_steps < 0) return fail(MDS_ERR_INVALID_ARGUMENT, "n_steps=%d < 0", n_steps);
    char* base = static_cast<char*>(plan->workspace);
    const BatchProblem* probs = reinterpret_cast<const BatchProblem*>(base);
    unsigned long long* cursor = reinterpret_cast<unsigned long long*>(
        base + align_up(sizeof(BatchProblem) * (size_t)plan->count, 256));
    // grad L and L at the current x of every problem, then the fused update
    auto evaluate = [&](double mult, int kick, int drift) -> int {
        hipError_t err = launch_batch_sweep(plan->y_dtype, true, plan->max_d, probs, plan->count,
                                            plan->total_tiles, cursor, plan->tile_waves,
                                            plan->lds_bytes, plan->grid, stream);
        if (err != hipSuccess) return hip_fail(err, "batch sweep launch");
        err = launch_batch_finalize(probs, batch_blkmap(plan), plan->count, plan->elem_blocks,
                                    cursor, mult, kick, drift, stream);
        if (err != hipSuccess) return hip_fail(err, "batch finalize launch");
        return MDS_OK;
    };
    int st;
    // the same sequence as mds_leapfrog: half kick and drift (fused into the
    // first evaluation unless the gradient is cached), full steps, half kick
    const bool fuse_first = !cache_valid && n_steps > 0;
    if (!cache_valid && (st = evaluate(0.5, fuse_first ? 1 : 0, fuse_first ? 1 : 0))) return st;
    if (n_steps > 0 && !fuse_first) {
        hipError_t e = launch_batch_kick_drift(probs, batch_blkmap(plan), plan->count,
                                               plan->elem_blocks, 0.5, 1, stream);
        if (e != hipSuccess) return hip_fail(e, "batch kick launch");
    }
    for (int s = 1; s <= n_steps; ++s) {
        const bool last = (s == n_steps);
        if ((st = evaluate(last ? 0.5 : 1.0, 1, last ? 0 : 1))) return st;
    }
    return MDS_OK;
}

int mds_set_tile_trace(void* trace)
{
    if (!aligned(trace, 8)) return fail(MDS_ERR_INVALID_ARGUMENT, "trace misaligned");
    g_tile_trace = static_cast<unsigned long long*>(trace);
    return MDS_OK;
}

int mds_set_sweep_events(hipEvent_t before, hipEvent_t after)
{
    if ((before == nullptr) != (after == nullptr))
        return fail(MDS_ERR_INVALID_ARGUMENT, "set both events or neither");
    g_ev_before = before;
    g_ev_after = after;
    return MDS_OK;
}

}  // extern "C"
