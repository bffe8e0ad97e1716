// mds_sweep.inc.h -- the fused pair sweep: one pass over the strict lower
// triangle of Y that produces the per-tile partial sums of the log-likelihood
// (Eq. 2), of dL/dsigma, and of every gradient row (Eq. 9).
//
// Work decomposition (gfx950, 64-wide waves):
//   * a work-group owns a tile of `br` rows x `cw` = 64*wc columns and runs
//     wc x wr waves: wave (u, v) owns columns c*cw + 64u .. +63, one column j
//     per lane, and the v-th of wr equal groups of the tile's rows;
//   * the wave walks its rows i in order (wave-uniform, so x_i comes through
//     scalar loads) and reads Y[i][j0 .. j0+63]: 64 consecutive elements of
//     one row, a fully coalesced load of the lower triangle;
//   * each pair's gradient term goes to row j (+) and row i (-) -- each pair
//     is evaluated once.  The column side stays in the lane's registers for
//     the wave's rows.  The row side is a sum across the 64 lanes: the lanes
//     stage their terms of a few rows in LDS, then every (row, dimension)
//     output is summed by a small group of lanes reading the staged values
//     and finished by log2(group) exchanges;
//   * a wavefront whose pairs in a row all have delta/sigma beyond a skip
//     point branches over the special functions as a whole (no divergence);
//   * the column sums of the wr waves of a column group, and the row sums of
//     the wc waves of a row group, meet in LDS and are added in wave order;
//     column, row and scalar partials of the tile go to the workspace, and
//     the finalize kernel adds them in a fixed order.  No atomics: the result
//     is bitwise reproducible.
// The paper's GPU design (one thread per pair in 16x16 work-groups for the
// likelihood, 128 threads per row for the gradient, every pair twice) is
// replaced by this single fused triangle pass.
#pragma once

#include <hip/hip_ext.h>

#include "mds_internal.h"
#include "mds_math.h"

namespace mds {

template <typename T>
__device__ __forceinline__ T shfl_xor_t(T v, int m)
{
    return __shfl_xor(v, m, kWave);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

// Per-pair arithmetic.  T = double: everything in FP64.  T = float: the
// difference x_i - x_j is formed in FP64 and rounded once (near-duplicate
// points would otherwise lose their distance to cancellation), the rest is
// FP32.
template <typename T>
struct PairConsts {
    T inv_sigma, inv_s2, half_inv_s2, inv_s3;
};

template <typename T>
__device__ __forceinline__ PairConsts<T> pair_consts(double sigma)
{
    PairConsts<T> c;
    const double is = 1.0 / sigma;
    c.inv_sigma = (T)is;
    c.inv_s2 = (T)(is * is);
    c.half_inv_s2 = (T)(0.5 * is * is);
    c.inv_s3 = (T)(is * is * is);
    return c;
}

template <typename T>
__device__ __forceinline__ T min_normal();
template <>
__device__ __forceinline__ double min_normal<double>()
{
    return 2.2250738585072014e-308;
}
template <>
__device__ __forceinline__ float min_normal<float>()
{
    return 1.17549435e-38f;
}

template <typename T>
__device__ __forceinline__ T rsqrt_t(T x);
template <>
__device__ __forceinline__ double rsqrt_t<double>(double x)
{
    return rsqrt_f64(x);
}
template <>
__device__ __forceinline__ float rsqrt_t<float>(float x)
{
    return __builtin_amdgcn_rsqf(x);
}

// both rows of a two-row step
template <typename T>
__device__ __forceinline__ void trunc_terms2(T t1, T t2, T& l1, T& m1, T& l2, T& m2)
{
    trunc_terms_f32(t1, l1, m1);
    trunc_terms_f32(t2, l2, m2);
}
template <>
__device__ __forceinline__ void trunc_terms2<double>(double t1, double t2, double& l1,
                                                     double& m1, double& l2, double& m2)
{
    trunc_terms2_f64(t1, t2, l1, m1, l2, m2);
}

template <typename T>
__device__ __forceinline__ void trunc_terms(T t, T& lnphi, T& mills);
template <>
__device__ __forceinline__ void trunc_terms<double>(double t, double& lnphi, double& mills)
{
    trunc_terms_f64(t, lnphi, mills);
}
template <>
__device__ __forceinline__ void trunc_terms<float>(float t, float& lnphi, float& mills)
{
    trunc_terms_f32(t, lnphi, mills);
}

// Per-pair quantities computed before the special functions.
template <typename T, int D>
struct PairGeom {
    T dl[D];   // x_i - x_j
    T delta;   // |x_i - x_j|
    T rinv;    // 1/delta (0 for a coincident pair)
    T t;       // delta / sigma
    T res;     // y - delta
    bool ok;   // an observed pair of the strict lower triangle
};

// Skip point of the truncation terms.  For t >= T, 0 <= -ln Phi(t) <=
// 2 Phi(-T) and phi(t)/Phi(t) <= 2 phi(T): below 2.3e-19 and 2.1e-18 for the
// FP64 sweep (T = 9), below 8.1e-11 and 5.4e-10 for the FP32 sweep (T = 6.5),
// each far under the rounding of the pair's other terms in that precision.
template <typename T>
__device__ __forceinline__ T skip_t();
template <>
__device__ __forceinline__ double skip_t<double>()
{
    return 9.0;
}
template <>
__device__ __forceinline__ float skip_t<float>()
{
    return 6.5f;
}

// lanes per output in the row reduction: the largest power of two g with
// outputs * g <= 64
__host__ __device__ constexpr int reduce_group(int outputs)
{
    int g = 64;
    while (g > 1 && outputs * g > 64) g >>= 1;
    return g;
}

// One tile of one problem, processed by the whole work-group; `lds` is the
// work-group's dynamic LDS (sweep_lds_bytes).  Ends with a barrier, so the
// caller may reuse the LDS for the next tile straight away.
template <typename T, int D, bool GRAD>
__device__ __forceinline__ void sweep_tile(const SweepArgs& a, const int64_t tile, double* lds)
{
    constexpr int RB = sweep_stage_rows(D);
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int waves = blockDim.x / kWave;
    const int br = a.br, cw = a.cw, wc = a.wc;
    const int wu = w % wc;  // this wave's column group

    int r, c;
    tile_coords(tile, a.nrb, br, cw, &r, &c);
    const WaveRows wv = wave_rows(a.n, br, cw, wc, a.wr, r, c, w, RB);
    const int64_t row0 = wv.row0, row1 = wv.row1;
    const int64_t j = wv.jw0 + lane;
    const bool colok = j < a.n;

    // LDS: [wc][br][D] tile row sums | [waves][4] scalars | [waves] staging
    // (rows of RB x (64 D + pad) elements, or a wave's 64 x D column sums)
    double* lrows = lds + (size_t)wu * br * D;
    double* lscal = lds + (size_t)wc * br * D;
    constexpr int SROW = kWave * D + kStagePadBytes / (int)sizeof(T);
    const size_t stage_bytes = sweep_stage_bytes(D, (int)sizeof(T));
    char* stage_base = reinterpret_cast<char*>(lscal + (size_t)waves * 4) + (size_t)w * stage_bytes;
    T* stage = reinterpret_cast<T*>(stage_base);
    // this wave's rows of the tile's row sums start at zero (rows it skips
    // hold no pair of its columns)
    if (GRAD)
        for (int k = lane; k < (int)(wv.rw1 - wv.rw0) * D; k += kWave)
            lrows[(wv.rw0 - row0) * D + k] = 0.0;

    double gj[D];
#pragma unroll
    for (int d = 0; d < D; ++d) gj[d] = 0.0;
    double acc_r = 0.0, acc_s = 0.0;
    int cnt = 0;

    if (wv.active) {
        double xj[D];
#pragma unroll
        for (int d = 0; d < D; ++d) xj[d] = colok ? a.x[j * a.ldx + d] : 0.0;
        const PairConsts<T> pc = pair_consts<T>(*a.sigma);
        const T* __restrict__ Y = static_cast<const T*>(a.y);

        // Y is prefetched two rows ahead, so each row's load has an iteration
        // of arithmetic to arrive.  The load is unconditional (lanes outside
        // the triangle discard the value through `ok`), so no branch splits
        // the wave and the wait before a row's first use leaves the two newer
        // loads in flight.  Rows are loaded strictly in order from ib0, and
        // the row pointer stops at the wave's last row rw1-1: every address
        // lies in rows [ib0, rw1) of the tile and in columns [0, n).  Row and
        // column indices fit 32 bits (N <= 2^30).
        const uint32_t jc = colok ? (uint32_t)j : 0u;
        const int j32 = (int)j;
        const int last_row = (int)(wv.rw1 - 1);
        const T* yrow = Y + wv.ib0 * a.ldy;
        int ynext = (int)wv.ib0;
        auto load_y = [&]() -> T {
            const T v = yrow[jc];
            if (ynext < last_row) yrow += a.ldy;
            ++ynext;
            return v;
        };
        // x_i is uniform across the wave and comes through scalar loads (X is
        // read-only during the sweep, so the constant address space is
        // valid); rows are visited in order, so its address advances by ldx
        const double* xrow = a.x + wv.ib0 * a.ldx;
        T pf0 = load_y(), pf1 = load_y();
        for (int64_t ib = wv.ib0; ib < wv.rw1; ib += RB) {
            T gjb[D];
#pragma unroll
            for (int d = 0; d < D; ++d) gjb[d] = T(0);
            T br_r = T(0), br_s = T(0);
            const int nq = (int)min((int64_t)RB, wv.rw1 - ib);

            // geometry of one pair row (row ib + q, this lane's column)
            auto geom = [&](const int q, const T yv, PairGeom<T, D>& g) {
                const int i = (int)(ib + q);
                const const_f64_ptr xi = (const_f64_ptr)xrow;
                xrow += a.ldx;
                g.ok = colok && (j32 < i) && !isnan(yv);
                T s2 = T(0);
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    g.dl[d] = (T)(xi[d] - xj[d]);
                    s2 = fma(g.dl[d], g.dl[d], s2);
                }
                // delta and 1/delta from one reciprocal square root.  A
                // coincident pair (s2 below the normal range) has no
                // direction: 1/delta is taken as 0, and delta = s2 *
                // rsqrt(min normal) is 0 for s2 = 0 (tiny otherwise)
                const T rs = rsqrt_t(fmax(s2, min_normal<T>()));
                g.delta = s2 * rs;
                g.rinv = (s2 >= min_normal<T>()) ? rs : T(0);
                g.t = g.delta * pc.inv_sigma;
                // a pair outside the sums gets y = delta: its residual is 0,
                // and with ln Phi = m = 0 (set by the caller) all its terms
                // vanish
                g.res = g.ok ? yv - g.delta : T(0);
            };
            // the pair's terms given ln Phi(t) and phi(t)/Phi(t) (both 0 for
            // a pair outside the sums)
            auto accum = [&](const int q, const PairGeom<T, D>& g, const T lnphi, const T mills) {
                const T res2 = g.res * g.res;
                br_r += fma(res2, pc.half_inv_s2, lnphi);
                if (GRAD) {
                    // w = (delta - y)/sigma^2 + m/sigma; the pair's term is
                    // w (x_i - x_j)/delta
                    const T wv_ = fma(mills, pc.inv_sigma, -g.res * pc.inv_s2);
                    const T coef = wv_ * g.rinv;
                    T* st = stage + (size_t)q * SROW + (size_t)lane * D;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        const T cd = coef * g.dl[d];
                        st[d] = -cd;
                        gjb[d] += cd;
                    }
                    br_s += fma(res2, pc.inv_s3, g.delta * pc.inv_s2 * mills);
                }
            };
            // observed pairs of a row in this wave (a wave-uniform count)
            auto count_ok = [&](const PairGeom<T, D>& g) {
                cnt += (int)__builtin_popcountll(__builtin_amdgcn_ballot_w64(g.ok));
            };
            // when no observed pair of the rows in this wave has t below the
            // skip point, the wave takes ln Phi = m = 0 and skips the special
            // functions (a wave-uniform branch; lanes never diverge)
            auto needs_tail = [&](const PairGeom<T, D>& g) { return g.ok && g.t < skip_t<T>(); };
            // two rows per step: their dependency chains interleave and they
            // share the special functions' coefficient loads
            int q = 0;
#pragma unroll 1
            for (; q + 1 < nq; q += 2) {
                const T ya = pf0, yb = pf1;
                pf0 = load_y();
                pf1 = load_y();
                PairGeom<T, D> ga, gb;
                geom(q, ya, ga);
                geom(q + 1, yb, gb);
                count_ok(ga);
                count_ok(gb);
                T la = T(0), ma = T(0), lb = T(0), mb = T(0);
                if (a.truncated && __builtin_amdgcn_ballot_w64(needs_tail(ga) || needs_tail(gb))) {
                    trunc_terms2<T>(ga.t, gb.t, la, ma, lb, mb);
                    la = ga.ok ? la : T(0);
                    ma = ga.ok ? ma : T(0);
                    lb = gb.ok ? lb : T(0);
                    mb = gb.ok ? mb : T(0);
                }
                accum(q, ga, la, ma);
                accum(q + 1, gb, lb, mb);
            }
            if (q < nq) {
                // the odd last row of the wave's rows
                const T ya = pf0;
                pf0 = pf1;
                pf1 = load_y();
                PairGeom<T, D> ga;
                geom(q, ya, ga);
                count_ok(ga);
                T la = T(0), ma = T(0);
                if (a.truncated && __builtin_amdgcn_ballot_w64(needs_tail(ga))) {
                    trunc_terms<T>(ga.t, la, ma);
                    la = ga.ok ? la : T(0);
                    ma = ga.ok ? ma : T(0);
                }
                accum(q, ga, la, ma);
            }
            acc_r += (double)br_r;
            if (GRAD) {
                acc_s += (double)br_s;
#pragma unroll
                for (int d = 0; d < D; ++d) gj[d] += (double)gjb[d];
                // transposed reduction of the staged rows: each (row,
                // dimension) output of the batch gets RG lanes; lane h of its
                // group adds the staged values of lanes h, h+RG, ..., then the
                // group combines by log2(RG) exchanges
                constexpr int NO = RB * D;
                constexpr int RG = reduce_group(NO);
                const int o = lane / RG, h = lane % RG;
                const int orow = o / D, odim = o % D;
                const bool live = o < NO && orow < nq;
                T sum = T(0);
                if (live) {
                    const T* src = stage + (size_t)orow * SROW + (size_t)h * D + odim;
#pragma unroll
                    for (int k = 0; k < kWave / RG; ++k) sum += src[(size_t)k * RG * D];
                }
#pragma unroll
                for (int m = RG / 2; m >= 1; m >>= 1) sum += shfl_xor_t(sum, m);
                if (live && h == 0) lrows[(ib - row0 + orow) * D + odim] = (double)sum;
            }
        }
    }

    const int wr = a.wr;
    double* cp = a.colpart + (((size_t)c * a.nrb + r) * cw + (size_t)wu * kWave + lane) * D;
    if (GRAD) {
        if (wr == 1) {
#pragma unroll
            for (int d = 0; d < D; ++d) cp[d] = gj[d];
        } else {
            // the wr waves of one column group add their column sums in LDS
            double* gs = reinterpret_cast<double*>(stage_base) + (size_t)lane * D;
#pragma unroll
            for (int d = 0; d < D; ++d) gs[d] = gj[d];
        }
    }
    acc_r = wave_sum(acc_r);
    acc_s = wave_sum(acc_s);
    // cnt is already the wave's total (a popcount of each row's ballot)
    if (lane == 0) {
        lscal[w * 4 + 0] = acc_r;
        lscal[w * 4 + 1] = acc_s;
        lscal[w * 4 + 2] = (double)cnt;
    }
    __syncthreads();
    if (GRAD) {
        if (wr > 1 && w < wc) {
            // wave (wu, 0) adds the column sums of waves (wu, 0..wr-1) in order
            double s[D];
#pragma unroll
            for (int d = 0; d < D; ++d) s[d] = 0.0;
            for (int v = 0; v < wr; ++v) {
                const double* gs = reinterpret_cast<const double*>(
                                       reinterpret_cast<const char*>(lscal + (size_t)waves * 4) +
                                       (size_t)(v * wc + wu) * stage_bytes) +
                                   (size_t)lane * D;
#pragma unroll
                for (int d = 0; d < D; ++d) s[d] += gs[d];
            }
#pragma unroll
            for (int d = 0; d < D; ++d) cp[d] = s[d];
        }
        // tile row sums: the column groups' copies added in order
        double* rp = a.rowpart + (size_t)tile * br * D;
        const int nrow = (int)(row1 - row0) * D;
        for (int k = threadIdx.x; k < nrow; k += blockDim.x) {
            double s = 0.0;
            for (int u = 0; u < wc; ++u) s += lds[(size_t)u * br * D + k];
            rp[k] = s;
        }
    }
    if (threadIdx.x == 0) {
        double sr = 0.0, ss = 0.0, sc = 0.0;
        for (int ww = 0; ww < waves; ++ww) {
            sr += lscal[ww * 4 + 0];
            ss += lscal[ww * 4 + 1];
            sc += lscal[ww * 4 + 2];
        }
        a.tscal[2 * tile + 0] = sr;
        a.tscal[2 * tile + 1] = ss;
        a.tcount[tile] = (uint32_t)sc;
    }
    __syncthreads();
}

template <typename T, int D, bool GRAD>
__global__ void __launch_bounds__(512) sweep_kernel(SweepArgs a)
{
    extern __shared__ double lds[];
    const bool traced = a.trace != nullptr;
    unsigned long long t0 = 0;
    if (traced) t0 = __builtin_amdgcn_s_memrealtime();
    sweep_tile<T, D, GRAD>(a, blockIdx.x, lds);
    if (traced) {
        // diagnostics: start and end clock (100 MHz) and HW_ID of each wave
        const unsigned long long t1 = __builtin_amdgcn_s_memrealtime();
        const unsigned long long hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);
        const int ln = threadIdx.x & (kWave - 1);
        if (ln < 3) {
            const unsigned long long v = ln == 0 ? t0 : (ln == 1 ? t1 : hw);
            a.trace[((size_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * 3 + ln] = v;
        }
    }
}

// Persistent sweep over the tiles of a batch of independent problems: each
// work-group takes the next global tile index from an atomic cursor until
// the batch is exhausted (every work-group reaches the exit), finds the
// problem that owns it, and runs that problem's tile with its own D.  Where
// a tile is processed never changes what it writes, so the results are those
// of the single-problem sweep, bit for bit.  MAXD bounds the D cases compiled
// in, so the register allocation follows the largest D of the batch.
template <typename T, bool GRAD, int MAXD>
__global__ void __launch_bounds__(512) batch_sweep_kernel(const BatchProblem* __restrict__ probs,
                                                          int32_t count, int64_t total_tiles,
                                                          unsigned long long* cursor)
{
    extern __shared__ double lds[];
    __shared__ int64_t next;
    for (;;) {
        if (threadIdx.x == 0) next = (int64_t)atomicAdd(cursor, 1ull);
        __syncthreads();
        const int64_t g = next;
        __syncthreads();
        if (g >= total_tiles) break;
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (probs[mid].tile_base <= g)
                lo = mid;
            else
                hi = mid - 1;
        }
        const BatchProblem& P = probs[lo];
        const SweepArgs a = P.sweep;
        const int64_t tile = g - P.tile_base;
        switch (P.d) {
            case 1: sweep_tile<T, 1, GRAD>(a, tile, lds); break;
            case 2: sweep_tile<T, 2, GRAD>(a, tile, lds); break;
            case 3: if constexpr (MAXD >= 3) sweep_tile<T, 3, GRAD>(a, tile, lds); break;
            case 4: if constexpr (MAXD >= 4) sweep_tile<T, 4, GRAD>(a, tile, lds); break;
            case 5: if constexpr (MAXD >= 5) sweep_tile<T, 5, GRAD>(a, tile, lds); break;
            case 6: if constexpr (MAXD >= 6) sweep_tile<T, 6, GRAD>(a, tile, lds); break;
            case 7: if constexpr (MAXD >= 7) sweep_tile<T, 7, GRAD>(a, tile, lds); break;
            default: if constexpr (MAXD >= 8) sweep_tile<T, 8, GRAD>(a, tile, lds); break;
        }
    }
}

// smallest compiled bound that covers max_d
inline int batch_maxd_bucket(int max_d) { return max_d <= 2 ? 2 : (max_d <= 4 ? 4 : (max_d <= 6 ? 6 : 8)); }

template <typename T, bool GRAD>
hipError_t launch_batch_sweep_g(int maxd, const BatchProblem* probs, int32_t count,
                                int64_t total_tiles, unsigned long long* cursor, dim3 g, dim3 b,
                                size_t lds, hipStream_t s)
{
    switch (batch_maxd_bucket(maxd)) {
        case 2:
            hipLaunchKernelGGL((batch_sweep_kernel<T, GRAD, 2>), g, b, lds, s, probs, count,
                               total_tiles, cursor);
            break;
        case 4:
            hipLaunchKernelGGL((batch_sweep_kernel<T, GRAD, 4>), g, b, lds, s, probs, count,
                               total_tiles, cursor);
            break;
        case 6:
            hipLaunchKernelGGL((batch_sweep_kernel<T, GRAD, 6>), g, b, lds, s, probs, count,
                               total_tiles, cursor);
            break;
        default:
            hipLaunchKernelGGL((batch_sweep_kernel<T, GRAD, 8>), g, b, lds, s, probs, count,
                               total_tiles, cursor);
            break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_sweep_t(bool grad, int maxd, const BatchProblem* probs, int32_t count,
                                int64_t total_tiles, unsigned long long* cursor, int waves,
                                size_t lds, int grid, hipStream_t s)
{
    if (total_tiles == 0) return hipSuccess;
    const dim3 g((unsigned)grid), b((unsigned)(waves * kWave));
    return grad ? launch_batch_sweep_g<T, true>(maxd, probs, count, total_tiles, cursor, g, b,
                                                lds, s)
                : launch_batch_sweep_g<T, false>(maxd, probs, count, total_tiles, cursor, g, b,
                                                 lds, s);
}

template <typename T, bool GRAD, int MAXD>
int occupancy_of(int waves, size_t lds)
{
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nb, batch_sweep_kernel<T, GRAD, MAXD>, waves * kWave, lds);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

template <typename T>
int batch_sweep_blocks_per_cu(bool grad, int maxd, int waves, size_t lds)
{
    switch (batch_maxd_bucket(maxd)) {
        case 2: return grad ? occupancy_of<T, true, 2>(waves, lds) : occupancy_of<T, false, 2>(waves, lds);
        case 4: return grad ? occupancy_of<T, true, 4>(waves, lds) : occupancy_of<T, false, 4>(waves, lds);
        case 6: return grad ? occupancy_of<T, true, 6>(waves, lds) : occupancy_of<T, false, 6>(waves, lds);
        default: return grad ? occupancy_of<T, true, 8>(waves, lds) : occupancy_of<T, false, 8>(waves, lds);
    }
}

template <typename T>
hipError_t launch_sweep_t(int d, bool grad, const Tiling& t, const SweepArgs& a, hipStream_t s,
                          hipEvent_t start, hipEvent_t stop)
{
    if (t.ntiles == 0) return hipSuccess;
    const dim3 grid((unsigned)t.ntiles), block((unsigned)(t.waves * kWave));
    const size_t lds = sweep_lds_bytes(t, d);
    const bool timed = start || stop;
#define MDS_SWEEP_LAUNCH(DD, G)                                                               \
    if (timed)                                                                                \
        hipExtLaunchKernelGGL((sweep_kernel<T, DD, G>), grid, block, lds, s, start, stop, 0,  \
                              a);                                                             \
    else                                                                                      \
        hipLaunchKernelGGL((sweep_kernel<T, DD, G>), grid, block, lds, s, a);
#define MDS_SWEEP_CASE(DD)            \
    case DD:                          \
        if (grad) {                   \
            MDS_SWEEP_LAUNCH(DD, true)  \
        } else {                      \
            MDS_SWEEP_LAUNCH(DD, false) \
        }                             \
        break;
    switch (d) {
        MDS_SWEEP_CASE(1)
        MDS_SWEEP_CASE(2)
        MDS_SWEEP_CASE(3)
        MDS_SWEEP_CASE(4)
        MDS_SWEEP_CASE(5)
        MDS_SWEEP_CASE(6)
        MDS_SWEEP_CASE(7)
        MDS_SWEEP_CASE(8)
        default:
            return hipErrorInvalidValue;
    }
#undef MDS_SWEEP_LAUNCH
#undef MDS_SWEEP_CASE
    return hipGetLastError();
}

}  // namespace mds
