// mds_lpd.hip -- log pointwise predictive density of held-out pairs (the
// model-selection part of Section 2): for each held-out pair, the log of the
// average over posterior draws of its truncated-normal density, summed over
// the pairs.
//
// The held-out pairs are first compacted into a list (row i, column j < i,
// y) in row-major order -- a count pass, an exclusive scan over the rows and
// a fill pass -- so that each draw costs O(pairs), not O(N^2).  Each draw
// then updates, per pair, a running log-sum-exp (largest term, sum of
// exp(l - largest)), and a last pass adds ln(average) over the pairs in a
// fixed order.
#include "mds_internal.h"
#include "mds_math.h"

namespace mds {
namespace {

constexpr int kRowThreads = 256;
constexpr int kScanThreads = 1024;
constexpr int kPartThreads = 256;

template <typename S>
__device__ __forceinline__ bool heldout_pair(const S* y, int64_t ld_y, const uint8_t* missing,
                                             int64_t ld_m, const uint8_t* heldout, int64_t ld_h,
                                             int64_t i, int64_t j)
{
    if (heldout[i * ld_h + j] == 0) return false;
    if (missing && missing[i * ld_m + j] != 0) return false;
    return !isnan(y[i * ld_y + j]);
}

// held-out pairs of row i (j < i)
template <typename S>
__global__ void __launch_bounds__(kRowThreads)
    heldout_count_kernel(const S* __restrict__ y, int64_t ld_y, const uint8_t* __restrict__ missing,
                         int64_t ld_m, const uint8_t* __restrict__ heldout, int64_t ld_h,
                         int64_t* __restrict__ row_count)
{
    const int64_t i = blockIdx.x;
    int c = 0;
    for (int64_t j = threadIdx.x; j < i; j += kRowThreads)
        c += heldout_pair(y, ld_y, missing, ld_m, heldout, ld_h, i, j) ? 1 : 0;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m, kWave);
    __shared__ int wsum[kRowThreads / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int q = 0; q < kRowThreads / kWave; ++q) t += wsum[q];
        row_count[i] = t;
    }
}

// in place: row_count -> exclusive row offsets; row n holds the total
__global__ void __launch_bounds__(kScanThreads)
    row_scan_kernel(int64_t n, int64_t* __restrict__ rows, int64_t* __restrict__ total)
{
    __shared__ int64_t part[kScanThreads];
    const int t = threadIdx.x;
    const int64_t chunk = (n + kScanThreads - 1) / kScanThreads;
    const int64_t r0 = min(n, (int64_t)t * chunk), r1 = min(n, r0 + chunk);
    int64_t s = 0;
    for (int64_t r = r0; r < r1; ++r) s += rows[r];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int q = 0; q < kScanThreads; ++q) {
            const int64_t v = part[q];
            part[q] = run;
            run += v;
        }
        rows[n] = run;
        *total = run;
    }
    __syncthreads();
    int64_t run = part[t];
    for (int64_t r = r0; r < r1; ++r) {
        const int64_t v = rows[r];
        rows[r] = run;
        run += v;
    }
}

// writes the held-out pairs of row i at its offset, in column order
template <typename S>
__global__ void __launch_bounds__(kRowThreads)
    heldout_fill_kernel(const S* __restrict__ y, int64_t ld_y, const uint8_t* __restrict__ missing,
                        int64_t ld_m, const uint8_t* __restrict__ heldout, int64_t ld_h,
                        const int64_t* __restrict__ row_off, int64_t capacity,
                        int32_t* __restrict__ pi, int32_t* __restrict__ pj, double* __restrict__ py)
{
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    __shared__ int wcount[kRowThreads / kWave];
    int64_t base = row_off[i];
    for (int64_t j0 = 0; j0 < i; j0 += kRowThreads) {
        const int64_t j = j0 + threadIdx.x;
        const bool keep = j < i && heldout_pair(y, ld_y, missing, ld_m, heldout, ld_h, i, j);
        const uint64_t mask = __builtin_amdgcn_ballot_w64(keep);
        const int before = __builtin_popcountll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[w] = __builtin_popcountll(mask);
        __syncthreads();
        int wbase = 0, all = 0;
        for (int q = 0; q < kRowThreads / kWave; ++q) {
            wbase += (q < w) ? wcount[q] : 0;
            all += wcount[q];
        }
        const int64_t k = base + wbase + before;
        if (keep && k < capacity) {
            pi[k] = (int32_t)i;
            pj[k] = (int32_t)j;
            py[k] = (double)y[i * ld_y + j];
        }
        base += all;
        __syncthreads();
    }
}

// per pair: l = ln p(y | delta, sigma) of the truncated normal for each of
// n_draws draws (draw s: x at xs + s * xstride, sigma = sigmas[s]), folded
// in draw order into the running log-sum-exp (acc[2k] = largest term,
// acc[2k+1] = sum of exp(l - largest)); `first` starts the sums with the
// first draw.  The state stays in registers across the draws, so a call with
// S draws reads and writes it once instead of S times.  Each thread takes
// lpd_pairs(S == 1) pairs (one block covers 256 times that many consecutive pairs,
// lane-strided so every load is coalesced), so ln sigma and 1/sigma are
// formed once per thread and draw.  A wavefront whose pairs all have
// delta/sigma >= 9 takes ln Phi = 0 (|ln Phi(t)| < 2.3e-19 there, far below
// the rounding of l).  The arithmetic of a draw does not depend on how the
// draws are grouped into calls: S calls of one draw and one call of S draws
// give the same bits.
// Pairs per thread (even: the special functions take two pairs at a time).
// One draw per pass streams the pair list and the state: two pairs per thread
// give twice the work-groups to hide memory latency (7% faster than four at
// 1.24 M pairs).  Several draws per pass are arithmetic-bound: four pairs per
// thread share ln sigma and 1/sigma of each draw (6% faster than two).
constexpr int lpd_pairs(bool one) { return one ? 2 : 4; }
static_assert(lpd_pairs(true) % 2 == 0 && lpd_pairs(false) % 2 == 0, "pairs per thread");
constexpr int kLpdThreads = 256;

template <int D, bool ONE>
__global__ void __launch_bounds__(kLpdThreads)
    lpd_accumulate_kernel(int64_t m, const int32_t* __restrict__ pi, const int32_t* __restrict__ pj,
                          const double* __restrict__ py, const double* __restrict__ xs,
                          int64_t ldx, int64_t xstride, const double* __restrict__ sigmas,
                          int32_t n_draws, double* __restrict__ acc, int first)
{
    constexpr double kLnSqrt2Pi = 0.91893853320467274178;
    constexpr int kLpdPairs = lpd_pairs(ONE);
    const int64_t base = (int64_t)blockIdx.x * (kLpdThreads * kLpdPairs) + threadIdx.x;
    int64_t ii[kLpdPairs], jj[kLpdPairs];
    double yv[kLpdPairs], mx[kLpdPairs], sm[kLpdPairs];
#pragma unroll
    for (int u = 0; u < kLpdPairs; ++u) {
        const int64_t k = base + (int64_t)u * kLpdThreads;
        // a lane past the end works on the last pair and stores nothing
        const int64_t kk = k < m ? k : m - 1;
        ii[u] = pi[kk];
        jj[u] = pj[kk];
        yv[u] = py[kk];
        mx[u] = first ? 0.0 : acc[2 * kk];
        sm[u] = first ? 0.0 : acc[2 * kk + 1];
    }
    // ONE: a single draw, with the loop known to run once (same arithmetic)
    const int32_t draws = ONE ? 1 : n_draws;
    const tab64_ptr tb = tab64();
    for (int s = 0; s < draws; ++s) {
        const double sigma = sigmas[s];
        const double inv_sigma = 1.0 / sigma;
        const double c0 = -kLnSqrt2Pi - log(sigma);
        const double* x = xs + (int64_t)s * xstride;
        const bool start = first && s == 0;
        double z[kLpdPairs], t[kLpdPairs];
#pragma unroll
        for (int u = 0; u < kLpdPairs; ++u) {
            double s2 = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const double diff = x[ii[u] * ldx + d] - x[jj[u] * ldx + d];
                s2 = fma(diff, diff, s2);
            }
            const double delta = sqrt(s2);
            z[u] = (yv[u] - delta) * inv_sigma;
            t[u] = delta * inv_sigma;
        }
        // ln Phi(t) two pairs at a time: skipped by the whole wave when every
        // t is past the skip point (9), in its far-range forms when every t
        // is at or past kFarT, else in its full-range forms
#pragma unroll
        for (int u = 0; u < kLpdPairs; u += 2) {
            double lp0 = 0.0, lp1 = 0.0, m0, m1;
            if (__builtin_amdgcn_ballot_w64(t[u] < 9.0) | __builtin_amdgcn_ballot_w64(t[u + 1] < 9.0)) {
                if ((__builtin_amdgcn_ballot_w64(t[u] < kFarT) |
                     __builtin_amdgcn_ballot_w64(t[u + 1] < kFarT)) == 0)
                    trunc_terms2_far_f64(t[u], t[u + 1], lp0, m0, lp1, m1, tb);
                else
                    trunc_terms2_f64(t[u], t[u + 1], lp0, m0, lp1, m1, tb);
            }
            const double lp[2] = {lp0, lp1};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int v = u + h;
                const double l = c0 - 0.5 * z[v] * z[v] - lp[h];
                // running log-sum-exp: one exp of -|l - largest| serves both
                // cases
                if (start) {
                    mx[v] = l;
                    sm[v] = 1.0;
                } else {
                    const double dl = l - mx[v];
                    const double e = exp(-fabs(dl));
                    if (dl > 0.0) {
                        sm[v] = sm[v] * e + 1.0;
                        mx[v] = l;
                    } else {
                        sm[v] += e;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < kLpdPairs; ++u) {
        const int64_t k = base + (int64_t)u * kLpdThreads;
        if (k < m) {
            acc[2 * k] = mx[u];
            acc[2 * k + 1] = sm[u];
        }
    }
}

// lpd = sum_k [acc_max + ln(acc_sum) - ln S], in two passes of fixed
// order: block b sums its contiguous share of the pairs (compensated
// per-thread sums, then a tree) into part[b]; one block adds the parts
__global__ void __launch_bounds__(kPartThreads)
    lpd_partial_kernel(int64_t m, const double* __restrict__ acc, double log_draws,
                       double* __restrict__ part)
{
    __shared__ double ps[kPartThreads];
    const int t = threadIdx.x;
    const int64_t chunk = (m + gridDim.x - 1) / gridDim.x;
    const int64_t k0 = (int64_t)blockIdx.x * chunk, k1 = min(m, k0 + chunk);
    double s = 0.0, c = 0.0;
    for (int64_t k = k0 + t; k < k1; k += kPartThreads) {
        const double v = acc[2 * k] + log(acc[2 * k + 1]) - log_draws;
        const double u = s + v;
        c += (fabs(s) >= fabs(v)) ? (s - u) + v : (v - u) + s;
        s = u;
    }
    ps[t] = s + c;
    __syncthreads();
    for (int h = kPartThreads / 2; h > 0; h >>= 1) {
        if (t < h) ps[t] += ps[t + h];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = ps[0];
}

__global__ void __launch_bounds__(kLpdMaxParts)
    lpd_sum_parts_kernel(int parts, const double* __restrict__ part, double* __restrict__ out)
{
    __shared__ double ps[kLpdMaxParts];
    const int t = threadIdx.x;
    ps[t] = t < parts ? part[t] : 0.0;
    __syncthreads();
    for (int h = kLpdMaxParts / 2; h > 0; h >>= 1) {
        if (t < h) ps[t] += ps[t + h];
        __syncthreads();
    }
    if (t == 0) *out = ps[0];
}

}  // namespace

hipError_t launch_heldout_count(const void* y, int dt, int64_t ld_y, const uint8_t* missing,
                                int64_t ld_m, const uint8_t* heldout, int64_t ld_h, int64_t n,
                                int64_t* rows, int64_t* total, hipStream_t s)
{
    if (n > 0) {
        if (dt == 0)
            hipLaunchKernelGGL((heldout_count_kernel<double>), dim3((unsigned)n), dim3(kRowThreads),
                               0, s, (const double*)y, ld_y, missing, ld_m, heldout, ld_h, rows);
        else
            hipLaunchKernelGGL((heldout_count_kernel<float>), dim3((unsigned)n), dim3(kRowThreads),
                               0, s, (const float*)y, ld_y, missing, ld_m, heldout, ld_h, rows);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(row_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, n, rows, total);
    return hipGetLastError();
}

hipError_t launch_heldout_fill(const void* y, int dt, int64_t ld_y, const uint8_t* missing,
                               int64_t ld_m, const uint8_t* heldout, int64_t ld_h, int64_t n,
                               const int64_t* rows, int64_t capacity, int32_t* pi, int32_t* pj,
                               double* py, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (dt == 0)
        hipLaunchKernelGGL((heldout_fill_kernel<double>), dim3((unsigned)n), dim3(kRowThreads), 0,
                           s, (const double*)y, ld_y, missing, ld_m, heldout, ld_h, rows, capacity,
                           pi, pj, py);
    else
        hipLaunchKernelGGL((heldout_fill_kernel<float>), dim3((unsigned)n), dim3(kRowThreads), 0,
                           s, (const float*)y, ld_y, missing, ld_m, heldout, ld_h, rows, capacity,
                           pi, pj, py);
    return hipGetLastError();
}

hipError_t launch_lpd_accumulate(int64_t m, const int32_t* pi, const int32_t* pj,
                                 const double* py, int d, const double* xs, int64_t ldx,
                                 int64_t xstride, const double* sigmas, int32_t n_draws,
                                 double* acc, int first, hipStream_t s)
{
    if (m == 0 || n_draws == 0) return hipSuccess;
    const int64_t per_block = (int64_t)kLpdThreads * lpd_pairs(n_draws == 1);
    const dim3 grid((unsigned)((m + per_block - 1) / per_block)), block(kLpdThreads);
#define MDS_LPD_CASE(DD)                                                                     \
    case DD:                                                                                 \
        if (n_draws == 1)                                                                    \
            hipLaunchKernelGGL((lpd_accumulate_kernel<DD, true>), grid, block, 0, s, m, pi, pj,   \
                               py, xs, ldx, xstride, sigmas, n_draws, acc, first);           \
        else                                                                                 \
            hipLaunchKernelGGL((lpd_accumulate_kernel<DD, false>), grid, block, 0, s, m, pi, pj,  \
                               py, xs, ldx, xstride, sigmas, n_draws, acc, first);           \
        break;
    switch (d) {
        MDS_LPD_CASE(1)
        MDS_LPD_CASE(2)
        MDS_LPD_CASE(3)
        MDS_LPD_CASE(4)
        MDS_LPD_CASE(5)
        MDS_LPD_CASE(6)
        MDS_LPD_CASE(7)
        MDS_LPD_CASE(8)
        default:
            return hipErrorInvalidValue;
    }
#undef MDS_LPD_CASE
    return hipGetLastError();
}

static int lpd_parts(int64_t m)
{
    const int64_t p = (m + 8 * kPartThreads - 1) / (8 * kPartThreads);
    return (int)max((int64_t)1, min((int64_t)kLpdMaxParts, p));
}

hipError_t launch_lpd_finalize(int64_t m, const double* acc, int64_t n_draws, double* part,
                               double* out, hipStream_t s)
{
    const int parts = lpd_parts(m);
    hipLaunchKernelGGL(lpd_partial_kernel, dim3(parts), dim3(kPartThreads), 0, s, m, acc,
                       log((double)n_draws), part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lpd_sum_parts_kernel, dim3(1), dim3(kLpdMaxParts), 0, s, parts, part, out);
    return hipGetLastError();
}

}  // namespace mds
