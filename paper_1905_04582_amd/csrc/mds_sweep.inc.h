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
//     and finished by log2(group) DPP lane exchanges;
//   * a wavefront whose pairs in two rows all have delta/sigma beyond a skip
//     point branches over the special functions as a whole (no divergence),
//     and the pair then adds one product to the wave's sums: the residual
//     square, which both the likelihood and dL/dsigma scale by a power of
//     1/sigma once per wave, and its gradient coefficient (scaled by
//     1/sigma^2 once per staging batch in FP32, once per walk in FP64); in
//     FP64 a wavefront whose pairs in
//     two rows all have delta/sigma >= 3 takes shorter far-range forms of the
//     special functions;
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

#include <type_traits>

#include "mds_internal.h"
#include "mds_math.h"
#include "mds_wave.h"

namespace mds {

// Per-pair arithmetic.  T = double: everything in FP64.  T = float: the
// difference x_i - x_j is formed in FP64 and rounded once (near-duplicate
// points would otherwise lose their distance to cancellation), the rest is
// FP32.
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

// both rows of a two-row step (`tb`: the FP64 coefficient tables)
template <typename T>
__device__ __forceinline__ void trunc_terms2(T t1, T t2, T& l1, T& m1, T& l2, T& m2, tab64_ptr)
{
    trunc_terms_f32(t1, l1, m1);
    trunc_terms_f32(t2, l2, m2);
}
template <>
__device__ __forceinline__ void trunc_terms2<double>(double t1, double t2, double& l1,
                                                     double& m1, double& l2, double& m2,
                                                     tab64_ptr tb)
{
    trunc_terms2_f64(t1, t2, l1, m1, l2, m2, tb);
}

// Skip point of the truncation terms.  For t >= T, 0 <= -ln Phi(t) <=
// 2 Phi(-T) and phi(t)/Phi(t) <= 2 phi(T): below 2.3e-19 and 2.1e-18 for the
// FP64 sweep (T = 9), below 8.1e-11 and 5.4e-10 for the FP32 sweep (T = 6.5),
// each far under the rounding of the pair's other terms in that precision.
// The sweep compares the squared distance with (T sigma)^2, so a pair within
// rounding of the skip point may fall on either side.
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

// One element of Y through a buffer resource: lane byte offset `voff`, row
// byte offset `soff` (uniform).
template <typename T>
__device__ __forceinline__ T load_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ double load_buf<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                   uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float load_buf<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                 uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
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
    const int wu = w & (wc - 1);  // this wave's column group (wc is a power of two)

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
    // the wave's sums over its pairs: A = sum (y - delta)^2, Lsum = sum ln Phi(t),
    // Msum = sum delta phi(t)/Phi(t); the tile's r and dsigma sums follow from
    // them (r = A / (2 sigma^2) + Lsum, dsigma terms = A / sigma^3 + Msum /
    // sigma^2), so a pair past the skip point adds one product to them
    double acc_A = 0.0, acc_L = 0.0, acc_M = 0.0;
    int cnt = 0;
    // sigma is read-only for the launch: a scalar load
    const double sig = *(const_f64_ptr)a.sigma;
    const double inv_s = 1.0 / sig;
    const double inv_s2 = inv_s * inv_s;

    if (wv.active) {
        double xj[D];
#pragma unroll
        for (int d = 0; d < D; ++d) xj[d] = colok ? a.x[j * a.ldx + d] : 0.0;
        const T sigT = (T)sig, inv_sT = (T)inv_s;
        // skip test on the squared distance: s2 >= (skip point * sigma)^2
        // means t >= the skip point (to the rounding of the bound).  The
        // model without truncation has no ln Phi and m terms: a negative
        // bound sends every step past them.
        const double tb = (double)skip_t<T>() * sig;
        const T thr2 = a.truncated ? (T)(tb * tb) : T(-1);
        // FP64: a step whose pairs all lie at t >= kFarT takes the shorter
        // far-range forms of the special functions
        const double tf = kFarT * sig;
        const T thrf = (T)(tf * tf);
        const T* __restrict__ Y = static_cast<const T*>(a.y);
        // the FP64 special functions' coefficient tables, addressed once
        const tab64_ptr ctab = sizeof(T) == 8 ? tab64() : nullptr;

        // Y is read two steps (four rows) ahead of use into two register
        // pairs that alternate, so each load has two steps of arithmetic to
        // arrive and no value is copied between registers.  Loads are
        // unconditional (lanes outside the triangle discard the value), and
        // rows are loaded strictly in order from ib0 with the row pointer
        // stopping at the wave's last row rw1-1: every address lies in rows
        // [ib0, rw1) of the tile and in columns [0, n).  Row and column
        // indices fit 32 bits (N <= 2^30); so does a lane's byte offset in a
        // row (the N^2 elements of Y must fit the device).
        const uint32_t joff = (colok ? (uint32_t)j : 0u) * (uint32_t)sizeof(T);
        const int j32 = (int)j;
        const uint64_t colmask = __builtin_amdgcn_ballot_w64(colok);
        const int ib0 = (int)wv.ib0, rw1 = (int)wv.rw1;
        const int last_row = rw1 - 1;
        // a buffer resource at the wave's first row: the row's byte offset is
        // a scalar operand and the lane's a fixed vector one, so a load costs
        // no vector address arithmetic (the host checks that the offsets of
        // a tile's rows fit 31 bits)
        const __amdgpu_buffer_rsrc_t yres = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<T*>(Y + wv.ib0 * a.ldy), (short)0, 0x7fffffff, 0x00020000);
        const uint32_t ystep = (uint32_t)a.ldy * (uint32_t)sizeof(T);
        uint32_t yoff = 0;
        int ynext = ib0;
        auto load_y = [&]() -> T {
            const T v = load_buf<T>(yres, joff, yoff);
            if (ynext < last_row) yoff += ystep;
            ++ynext;
            return v;
        };
        // x_i is uniform across the wave and comes through scalar loads (X is
        // read-only during the sweep, so the constant address space is
        // valid); rows are visited in order, so its address advances by ldx
        // and, like Y's, stops at the wave's last row
        const double* xrow = a.x + wv.ib0 * a.ldx;
        int xnext = ib0;
        auto next_x = [&]() -> const_f64_ptr {
            const const_f64_ptr p = (const_f64_ptr)xrow;
            if (xnext < last_row) xrow += a.ldx;
            ++xnext;
            return p;
        };

        constexpr int NO = RB * D;
        constexpr int RG = reduce_group(NO);
        const int o = lane / RG, h = lane % RG;
        const int orow = o / D, odim = o % D;

        T gjb[D];
        T bA, bL, bM;
        auto batch_reset = [&]() {
#pragma unroll
            for (int d = 0; d < D; ++d) gjb[d] = T(0);
            bA = T(0);
            bL = T(0);
            bM = T(0);
        };
        // In FP32 the lane sums (bA, bL, bM, gjb) close into the FP64
        // accumulators at the end of each staging batch; in FP64 they are
        // those accumulators and run over the whole walk.
        constexpr bool BATCH_SUMS = sizeof(T) < sizeof(double);
        auto close_sums = [&]() {
            acc_A += (double)bA;
            acc_L += (double)bL;
            acc_M += (double)bM;
#pragma unroll
            for (int d = 0; d < D; ++d) gj[d] = fma((double)gjb[d], inv_s2, gj[d]);
        };
        // end of the staging batch of rows [b0, b0 + RB) (rows at or past rw1
        // are dead): every (row, dimension) output gets RG lanes -- lane h of
        // its group adds the staged values of lanes h, h+RG, ..., then the
        // group combines by log2(RG) exchanges
        auto batch_flush = [&](auto fast_tag, const int b0) {
            constexpr bool FAST = decltype(fast_tag)::value;
            if constexpr (BATCH_SUMS) close_sums();
            if (GRAD) {
                const bool live = o < NO && (FAST || b0 + orow < rw1);
                T sum = T(0);
                if (live) {
                    const T* src = stage + (size_t)orow * SROW + (size_t)h * D + odim;
                    sum = src[0];
#pragma unroll
                    for (int k = 1; k < kWave / RG; ++k) sum += src[(size_t)k * RG * D];
                }
                sum = group_sum<RG>(sum);
                if (live && h == 0) lrows[(b0 - row0 + orow) * D + odim] = (double)sum * inv_s2;
            }
            if constexpr (BATCH_SUMS) batch_reset();
        };
        batch_reset();

        // One step: rows i0 and i0 + 1, staged at positions q and q + 1 of
        // the batch.  FAST (a compile-time tag) is the walk of a wave whose
        // rows are whole iterations with x rows contiguous (ldx == D); the
        // general walk has dead rows (at or past rw1: no lane's pair counts,
        // their loads repeat the wave's last row).
        auto step = [&](auto fast_tag, const int i0, const int q, const T ya, const T yb) {
            constexpr bool FAST = decltype(fast_tag)::value;
            const bool live0 = FAST || i0 < rw1, live1 = FAST || i0 + 1 < rw1;
            const_f64_ptr xa, xb;
            if constexpr (FAST) {
                xa = (const_f64_ptr)xrow;
                xb = xa + D;
                xrow += 2 * D;
            } else {
                xa = next_x();
                xb = next_x();
            }
            T da[D], db[D];
            T s2a = T(0), s2b = T(0);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                da[d] = (T)(xa[d] - xj[d]);
                db[d] = (T)(xb[d] - xj[d]);
                s2a = fma(da[d], da[d], s2a);
                s2b = fma(db[d], db[d], s2b);
            }
            // observed pairs as wave masks: the lanes below the row (j < i),
            // of a present y, of a column inside the problem, on a live row.
            // Each compare feeds only its ballot, and a lane's condition is
            // then the mask's own bit (combined and counted by scalar
            // instructions, with no per-lane copy of the conditions)
            const uint64_t ma = __builtin_amdgcn_ballot_w64(j32 < i0) &
                                __builtin_amdgcn_ballot_w64(!isnan(ya)) &
                                colmask & (0ull - (uint64_t)live0);
            const uint64_t mb = __builtin_amdgcn_ballot_w64(j32 <= i0) &
                                __builtin_amdgcn_ballot_w64(!isnan(yb)) & colmask &
                                (0ull - (uint64_t)live1);
            cnt += (int)__builtin_popcountll(ma) + (int)__builtin_popcountll(mb);
            const bool oka = __builtin_amdgcn_inverse_ballot_w64(ma);
            const bool okb = __builtin_amdgcn_inverse_ballot_w64(mb);
            // any observed pair closer than the skip point sends the wave
            // through the special functions (the others' terms are masked)
            const uint64_t near = (__builtin_amdgcn_ballot_w64(s2a < thr2) & ma) |
                                  (__builtin_amdgcn_ballot_w64(s2b < thr2) & mb);
            // delta and 1/delta from one reciprocal square root of s2 clamped
            // to the smallest normal number.  A coincident pair (s2 = 0) gets
            // delta = 0 and a gradient term (coefficient) * (x_i - x_j) = 0;
            // below the normal range the clamp keeps 1/delta finite, and the
            // term stays below the residual in size, as it is at any distance
            const T rsa = rsqrt_t(fmax(s2a, min_normal<T>()));
            const T rsb = rsqrt_t(fmax(s2b, min_normal<T>()));
            // a pair outside the sums gets residual 0 (and, below, ln Phi =
            // m = 0): all its terms vanish
            const T ra = oka ? fma(-s2a, rsa, ya) : T(0);
            const T rb = okb ? fma(-s2b, rsb, yb) : T(0);
            bA = fma(ra, ra, bA);
            bA = fma(rb, rb, bA);
            // sigma^2 w (x_i - x_j)/delta = (m sigma - (y - delta)) (x_i -
            // x_j)/delta; far pairs (t past the skip point for every lane of
            // the wave) take m = ln Phi = 0 without evaluating them
            T ca = -ra * rsa, cb = -rb * rsb;
            if (near) {
                const T dla = s2a * rsa, dlb = s2b * rsb;
                T la, mla, lb, mlb;
                if constexpr (sizeof(T) == 8) {
                    if ((__builtin_amdgcn_ballot_w64(s2a < thrf) |
                         __builtin_amdgcn_ballot_w64(s2b < thrf)) == 0)
                        trunc_terms2_far_f64(dla * inv_sT, dlb * inv_sT, la, mla, lb, mlb, ctab);
                    else
                        trunc_terms2<T>(dla * inv_sT, dlb * inv_sT, la, mla, lb, mlb, ctab);
                } else {
                    trunc_terms2<T>(dla * inv_sT, dlb * inv_sT, la, mla, lb, mlb, ctab);
                }
                la = oka ? la : T(0);
                mla = oka ? mla : T(0);
                lb = okb ? lb : T(0);
                mlb = okb ? mlb : T(0);
                bL += la + lb;
                bM = fma(dla, mla, bM);
                bM = fma(dlb, mlb, bM);
                ca = fma(mla * sigT, rsa, ca);
                cb = fma(mlb * sigT, rsb, cb);
            }
            if (GRAD) {
                T* st = stage + (size_t)q * SROW + (size_t)lane * D;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    st[d] = -ca * da[d];
                    st[SROW + d] = -cb * db[d];
                    gjb[d] = fma(ca, da[d], gjb[d]);
                    gjb[d] = fma(cb, db[d], gjb[d]);
                }
            }
        };
        const std::true_type fast_walk;
        const std::false_type general_walk;

        // The fast walk: the wave's rows are a whole number of staging
        // batches of at least four rows and its x rows are contiguous, so no
        // row is dead and x of two rows is one scalar load.  Each iteration
        // prefetches the next four rows from one base offset, capped at the
        // wave's last four rows: the last iteration reads those again (its
        // values are never used) instead of rows past rw1.  Two steps of two
        // rows per iteration take the two register pairs in turn; a batch of
        // RB rows closes after RB/2 steps.
        constexpr int IT = RB > 4 ? RB : 4;
        const bool fast = ((rw1 - ib0) % IT == 0) && (a.ldx == D);
        if (fast) {
            const uint32_t ystep2 = 2 * ystep, ystep3 = 3 * ystep;
            const uint32_t ycap = (uint32_t)(rw1 - 4 - ib0) * ystep;
            T pa0 = load_buf<T>(yres, joff, 0), pa1 = load_buf<T>(yres, joff, ystep);
            // keep the issue order: the first pair is consumed first
            __builtin_amdgcn_sched_barrier(0);
            T pb0 = load_buf<T>(yres, joff, ystep2), pb1 = load_buf<T>(yres, joff, ystep3);
            uint32_t ynext = 4 * ystep;  // offset of the row after the loaded ones
            int q = 0;  // staging position of the iteration's first row
#pragma unroll 1
            for (int ib = ib0; ib < rw1; ib += 4) {
                const uint32_t yb = min(ynext, ycap);
                ynext += 4 * ystep;
                step(fast_walk, ib, q, pa0, pa1);
                pa0 = load_buf<T>(yres, joff, yb);
                pa1 = load_buf<T>(yres, joff, yb + ystep);
                if (RB == 2) batch_flush(fast_walk, ib);
                step(fast_walk, ib + 2, RB == 2 ? 0 : q + 2, pb0, pb1);
                pb0 = load_buf<T>(yres, joff, yb + ystep2);
                pb1 = load_buf<T>(yres, joff, yb + ystep3);
                q += 4;
                if (q >= RB) {
                    batch_flush(fast_walk, ib + 4 - RB);
                    q = 0;
                }
            }
        } else {
            // The general walk: four rows per iteration; rows past rw1 in the
            // last iteration are dead, and a batch the walk leaves open
            // closes after it.
            T pa0 = load_y(), pa1 = load_y();
            __builtin_amdgcn_sched_barrier(0);
            T pb0 = load_y(), pb1 = load_y();
            int q = 0;  // staging position of the next step
            int ib = ib0;
#pragma unroll 1
            for (; ib < rw1; ib += 4) {
                step(general_walk, ib, q, pa0, pa1);
                pa0 = load_y();
                pa1 = load_y();
                q += 2;
                if (q == RB) {
                    batch_flush(general_walk, ib + 2 - RB);
                    q = 0;
                }
                step(general_walk, ib + 2, q, pb0, pb1);
                pb0 = load_y();
                pb1 = load_y();
                q += 2;
                if (q == RB) {
                    batch_flush(general_walk, ib + 4 - RB);
                    q = 0;
                }
            }
            // (rows [ib - q, ib))
            if (q != 0) batch_flush(general_walk, ib - q);
        }
        if constexpr (!BATCH_SUMS) close_sums();
    }

    double acc_r = fma(acc_A, 0.5 * inv_s2, acc_L);
    double acc_s = fma(acc_A, inv_s2 * inv_s, acc_M * inv_s2);

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

// Waves per SIMD the register allocation must allow for D <= 2: four in
// FP64 (the LDS of four 4-wave work-groups per compute unit), seven in FP32;
// no bound above (the allocator's own choice).
template <typename T, int D>
constexpr int sweep_waves_per_simd() { return D > 2 ? 1 : (sizeof(T) == 8 ? 4 : 7); }
// The persistent batch kernel carries the problem lookup on top of the walk:
// in FP32 with D <= 2 it fits five waves per SIMD without spilling (at six
// or seven it spills).
template <typename T, int MAXD>
constexpr int batch_sweep_waves_per_simd()
{
    return (sizeof(T) == 4 && MAXD <= 2) ? 5 : sweep_waves_per_simd<T, MAXD>();
}

template <typename T, int D, bool GRAD>
__global__ void __launch_bounds__(512)
    __attribute__((amdgpu_waves_per_eu(sweep_waves_per_simd<T, D>()))) sweep_kernel(SweepArgs a)
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
__global__ void __launch_bounds__(512)
    __attribute__((amdgpu_waves_per_eu(batch_sweep_waves_per_simd<T, MAXD>()))) batch_sweep_kernel(const BatchProblem* __restrict__ probs,
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
