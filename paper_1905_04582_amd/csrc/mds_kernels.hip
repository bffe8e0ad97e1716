// mds_kernels.hip -- the kernels around the pair sweep: the deterministic
// finalize (partials -> gradient rows, L, dL/dsigma, fused leapfrog kick and
// drift), the Hamiltonian energy, the Y preparation and the elementwise
// special-function helper.
#include <type_traits>

#include "mds_internal.h"
#include "mds_math.h"
#include "mds_wave.h"

namespace mds {

hipError_t launch_sweep_f64(int d, bool grad, const Tiling& t, const SweepArgs& a, hipStream_t s,
                            hipEvent_t start, hipEvent_t stop);
hipError_t launch_sweep_f32(int d, bool grad, const Tiling& t, const SweepArgs& a, hipStream_t s,
                            hipEvent_t start, hipEvent_t stop);

hipError_t launch_batch_sweep_f64(bool grad, int maxd, const BatchProblem* probs, int32_t count,
                                 int64_t total_tiles, unsigned long long* cursor, int waves,
                                 size_t lds, int grid, hipStream_t s);
hipError_t launch_batch_sweep_f32(bool grad, int maxd, const BatchProblem* probs, int32_t count,
                                 int64_t total_tiles, unsigned long long* cursor, int waves,
                                 size_t lds, int grid, hipStream_t s);
int batch_sweep_blocks_per_cu_f64(bool grad, int maxd, int waves, size_t lds);
int batch_sweep_blocks_per_cu_f32(bool grad, int maxd, int waves, size_t lds);

hipError_t launch_sweep(int y_dtype, int d, bool grad, const Tiling& t, const SweepArgs& a,
                        hipStream_t s, hipEvent_t start, hipEvent_t stop)
{
    return y_dtype == 0 ? launch_sweep_f64(d, grad, t, a, s, start, stop)
                        : launch_sweep_f32(d, grad, t, a, s, start, stop);
}

hipError_t launch_batch_sweep(int y_dtype, bool grad, int maxd, const BatchProblem* probs,
                              int32_t count, int64_t total_tiles, unsigned long long* cursor,
                              int waves, size_t lds, int grid, hipStream_t s)
{
    return y_dtype == 0 ? launch_batch_sweep_f64(grad, maxd, probs, count, total_tiles, cursor,
                                                 waves, lds, grid, s)
                        : launch_batch_sweep_f32(grad, maxd, probs, count, total_tiles, cursor,
                                                 waves, lds, grid, s);
}

int batch_sweep_blocks_per_cu(int y_dtype, bool grad, int maxd, int waves, size_t lds)
{
    return y_dtype == 0 ? batch_sweep_blocks_per_cu_f64(grad, maxd, waves, lds)
                        : batch_sweep_blocks_per_cu_f32(grad, maxd, waves, lds);
}

// Finalize: one work-group per 64 consecutive gradient elements e = (k, d),
// plus one scalar work-group (the last one).  Element e owns a list of
// partials: the row-side partials of row k over the tiles of its row block,
// then the column-side partials over the tiles of its column block.  Wave w
// of kFinChunks adds list items w, w + kFinChunks, ... (64 consecutive
// elements per wave: coalesced reads), and wave 0 adds the kFinChunks chunk
// sums in chunk order.  Every order is fixed, so the result is reproducible.
constexpr int kFinChunks = 8;
constexpr int kFinUnroll = 16;  // partial loads in flight per lane
// The finalize streams partials with one round of loads per lane: its time is
// latency, so the register budget is held to six waves per SIMD (three
// work-groups per compute unit; at the default budget the batched kernel fit
// one).
constexpr int kFinWavesPerSimd = 6;

// The scalar part: L, dL/dsigma and dL/d(ln sigma) from the per-tile sums,
// by one work-group of kWave * kFinChunks threads in a fixed order: thread t
// adds tiles t, t + T, ... (loads issued in batches sized to the tile count),
// each wave sums its lanes by DPP exchanges (the pair counts are integers
// below 2^53, so their sums in FP64 are exact in any order), and thread 0
// adds the waves in order.  ln sigma and 1/sigma are
// formed while the loads are in flight.
__device__ void finalize_scalars(const FinalizeArgs& a, double scale)
{
    constexpr int T = kWave * kFinChunks;
    __shared__ double s[3][kFinChunks];
    const int t = threadIdx.x, w = t / kWave;
    const double sigma = *a.sigma;
    double sr = 0.0, ss = 0.0, sm = 0.0;
    const int64_t last = a.ntiles - 1;
    auto add_tiles = [&](auto batch) {
        constexpr int U = decltype(batch)::value;
        for (int64_t u = t; u < a.ntiles; u += U * T) {
            double r[U], q[U];
            uint32_t c[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int64_t v = min(u + (int64_t)k * T, last);
                r[k] = a.tscal[2 * v + 0];
                q[k] = a.tscal[2 * v + 1];
                c[k] = a.tcount[v];
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const bool in = u + (int64_t)k * T < a.ntiles;
                sr += in ? r[k] : 0.0;
                ss += in ? q[k] : 0.0;
                sm += in ? (double)c[k] : 0.0;
            }
        }
    };
    // (at most 8 tiles per batch: larger batches cost the element blocks of
    // the same kernel their occupancy)
    if (a.ntiles <= 4 * T)
        add_tiles(std::integral_constant<int, 4>());
    else
        add_tiles(std::integral_constant<int, 8>());
    const double ln_sigma = log(sigma), inv_sigma = 1.0 / sigma;
    sr = wave_sum(sr);
    ss = wave_sum(ss);
    sm = wave_sum(sm);
    if ((t & (kWave - 1)) == 0) {
        s[0][w] = sr;
        s[1][w] = ss;
        s[2][w] = sm;
    }
    __syncthreads();
    if (t == 0) {
        double r0 = 0.0, q0 = 0.0, m = 0.0;
        for (int k = 0; k < kFinChunks; ++k) {
            r0 += s[0][k];
            q0 += s[1][k];
            m += s[2][k];
        }
        const double L = (m > 0.0) ? -m * ln_sigma - r0 : 0.0;
        const double ds = (m > 0.0) ? (-m * inv_sigma + q0) * scale : 0.0;
        if (a.loglik) *a.loglik = L;
        if (a.dsigma) *a.dsigma = ds;
        if (a.dlogsigma) *a.dlogsigma = ds * sigma;
    }
}

// The gradient part for element block `blk` (64 consecutive elements).
// Indices are 32-bit: n D < 2^31 (the host bounds n through Y's leading
// dimension) and tile and row-block counts are below 2^31.
__device__ void finalize_elements(const FinalizeArgs& a, int D, int64_t blk, double scale)
{
    __shared__ double part[kFinChunks][kWave];
    const int lane = threadIdx.x % kWave;
    const int chunk = threadIdx.x / kWave;
    const uint32_t e = (uint32_t)blk * kWave + lane;
    const bool live = e < (uint32_t)(a.n * D);
    const int br = a.br, cw = a.cw;
    const int lbr = __builtin_ctz((unsigned)br), lcw = __builtin_ctz((unsigned)cw);

    double s = 0.0;
    uint32_t k = 0;
    int d = 0;
    if (live) {
        k = e / (uint32_t)D;
        d = (int)(e - k * (uint32_t)D);
        const int r = (int)(k >> lbr);
        const uint32_t roff = k & (uint32_t)(br - 1);
        const int64_t t0 = tiles_before(r, br, cw);
        const int nrow = (int)tiles_in_row_block(r, br, cw);
        const int c = (int)(k >> lcw);
        const uint32_t coff = k & (uint32_t)(cw - 1);
        const int rb0 = first_row_block_of_column(c, br, cw);
        const int total = nrow + (a.nrb - rb0);
        // The element's list: the row-side partials of row k over the nrow
        // tiles of its row block, then the column-side partials of column k
        // over row blocks rb0 .. nrb-1.  Chunk `chunk` adds items chunk,
        // chunk + kFinChunks, ... in list order.  Loads are unconditional
        // (index clamped into the list, an item past the end replaced by 0),
        // so each batch of loads -- row and column items alike -- is in
        // flight together.  The batch is 4, 8 or kFinUnroll loads, the
        // fewest that cover a chunk's items in one batch where that is
        // possible (the order of the additions is the same whatever the
        // batch).
        const double* rbase = a.rowpart + ((t0 * br + roff) * D + d);
        const double* cbase = a.colpart + ((((int64_t)c * a.nrb + rb0) * cw + coff) * D + d);
        const int64_t rstep = (int64_t)br * D, cstep = (int64_t)cw * D;
        auto add_items = [&](auto batch) {
            constexpr int U = decltype(batch)::value;
            for (int i0 = chunk; i0 < total; i0 += U * kFinChunks) {
                double v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int q = min(i0 + u * kFinChunks, total - 1);
                    v[u] = q < nrow ? rbase[q * rstep] : cbase[(q - nrow) * cstep];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) s += (i0 + u * kFinChunks < total) ? v[u] : 0.0;
            }
        };
        if (total <= 4 * kFinChunks)
            add_items(std::integral_constant<int, 4>());
        else if (total <= 8 * kFinChunks)
            add_items(std::integral_constant<int, 8>());
        else
            add_items(std::integral_constant<int, kFinUnroll>());
    }
    part[chunk][lane] = s;
    __syncthreads();
    if (chunk != 0 || !live) return;
    double tot = part[0][lane];
#pragma unroll
    for (int q = 1; q < kFinChunks; ++q) tot += part[q][lane];

    double g = tot * scale;
    if (a.prior) g -= (*a.prior) * a.x[k * a.ldx + d];
    if (a.grad) a.grad[k * a.ldg + d] = g;
    if (a.p) {
        const double eps = *a.step;
        double* pp = a.p + k * a.ldp + d;
        const double pn = *pp + a.kick_mult * eps * g;
        *pp = pn;
        if (a.drift) {
            const double im = a.inv_mass ? a.inv_mass[k * D + d] : 1.0;
            a.x[k * a.ldx + d] += eps * im * pn;
        }
    }
}

__global__ void __launch_bounds__(kWave * kFinChunks)
    __attribute__((amdgpu_waves_per_eu(kFinWavesPerSimd))) finalize_kernel(FinalizeArgs a, int D)
{
    const double scale = a.scale ? *a.scale : 1.0;
    if (blockIdx.x == gridDim.x - 1)
        finalize_scalars(a, scale);
    else
        finalize_elements(a, D, blockIdx.x, scale);
}

// Batched finalize: element blocks of every problem, then one scalar block
// per problem.  Also rewinds the persistent sweep's tile cursor for the next
// call (this kernel runs after the sweep on the same stream).
__global__ void __launch_bounds__(kWave * kFinChunks)
    __attribute__((amdgpu_waves_per_eu(kFinWavesPerSimd))) batch_finalize_kernel(const BatchProblem* __restrict__ probs,
                          const int32_t* __restrict__ blkmap, int32_t count, int64_t elem_blocks,
                          unsigned long long* cursor, double kick_mult, int kick, int drift)
{
    int64_t b = blockIdx.x;
    int k;
    if (b < elem_blocks) {
        // the block's problem from the map the batch set-up wrote (one load
        // instead of a search over the problem table)
        k = blkmap[b];
    } else {
        k = (int)(b - elem_blocks);
        if (k == 0 && threadIdx.x == 0) *cursor = 0ull;
    }
    const BatchProblem& P = probs[k];
    FinalizeArgs a = {};
    a.n = P.sweep.n;
    a.br = P.sweep.br;
    a.cw = P.sweep.cw;
    a.nrb = P.sweep.nrb;
    a.ntiles = P.ntiles;
    a.rowpart = P.sweep.rowpart;
    a.colpart = P.sweep.colpart;
    a.tscal = P.sweep.tscal;
    a.tcount = P.sweep.tcount;
    a.sigma = P.sweep.sigma;
    a.grad = P.grad;
    a.ldg = P.ldg;
    a.loglik = P.loglik;
    a.dsigma = P.dsigma;
    a.dlogsigma = P.dlogsigma;
    if (kick) {
        a.x = P.x;
        a.ldx = P.sweep.ldx;
        a.p = P.p;
        a.ldp = P.ldp;
        a.step = P.step;
        a.kick_mult = kick_mult;
        a.drift = drift;
    }
    const double scale = P.scale ? *P.scale : 1.0;
    if (b < elem_blocks)
        finalize_elements(a, P.d, b - P.blk_base, scale);
    else
        finalize_scalars(a, scale);
}

hipError_t launch_batch_finalize(const BatchProblem* probs, const int32_t* blkmap, int32_t count,
                                 int64_t elem_blocks, unsigned long long* cursor, double kick_mult,
                                 int kick, int drift, hipStream_t s)
{
    const unsigned nblk = (unsigned)(elem_blocks + count);
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(nblk), dim3(kWave * kFinChunks), 0, s, probs,
                       blkmap, count, elem_blocks, cursor, kick_mult, kick, drift);
    return hipGetLastError();
}

// one work-group of 64 threads per finalize element block (64 consecutive
// elements of one problem): p += kick_mult eps g, then x += eps p
__global__ void __launch_bounds__(kWave)
    batch_kick_drift_kernel(const BatchProblem* __restrict__ probs,
                            const int32_t* __restrict__ blkmap, double kick_mult, int drift)
{
    const int64_t b = blockIdx.x;
    const BatchProblem& P = probs[blkmap[b]];
    const int D = P.d;
    const int64_t e = (b - P.blk_base) * kWave + threadIdx.x;
    if (e >= P.sweep.n * D) return;
    const int64_t k = e / D;
    const int d = (int)(e - k * D);
    const double eps = *P.step;
    double* pp = P.p + k * P.ldp + d;
    const double pn = *pp + kick_mult * eps * P.grad[k * P.ldg + d];
    *pp = pn;
    if (drift) P.x[k * P.sweep.ldx + d] += eps * pn;
}

hipError_t launch_batch_kick_drift(const BatchProblem* probs, const int32_t* blkmap,
                                   int32_t count, int64_t elem_blocks, double kick_mult, int drift,
                                   hipStream_t s)
{
    (void)count;
    if (elem_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(batch_kick_drift_kernel, dim3((unsigned)elem_blocks), dim3(kWave), 0, s,
                       probs, blkmap, kick_mult, drift);
    return hipGetLastError();
}

hipError_t launch_finalize(int d, const FinalizeArgs& a, hipStream_t s)
{
    const int64_t nel = a.grad ? a.n * d : 0;
    const unsigned nblk = (unsigned)((nel + kWave - 1) / kWave) + 1;
    hipLaunchKernelGGL(finalize_kernel, dim3(nblk), dim3(kWave * kFinChunks), 0, s, a, d);
    return hipGetLastError();
}

// ---------------------------------------------------------- leapfrog ----

// p += mult * eps * g; then (drift) x += eps * M^-1 p.  Element-parallel.
__global__ void __launch_bounds__(256)
    kick_drift_kernel(int64_t n, int D, double* x, int64_t ldx, double* p, int64_t ldp,
                      const double* g, const double* inv_mass, const double* step, double mult,
                      int drift)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * D) return;
    const int64_t k = e / D;
    const int d = (int)(e - k * D);
    const double eps = *step;
    double* pp = p + k * ldp + d;
    const double pn = *pp + mult * eps * g[e];
    *pp = pn;
    if (drift) x[k * ldx + d] += eps * (inv_mass ? inv_mass[e] : 1.0) * pn;
}

hipError_t launch_kick_drift(int64_t n, int d, double* x, int64_t ldx, double* p, int64_t ldp,
                             const double* g, const double* inv_mass, const double* step,
                             double mult, int drift, hipStream_t s)
{
    if (n * d == 0) return hipSuccess;
    const unsigned nblk = (unsigned)((n * d + 255) / 256);
    hipLaunchKernelGGL(kick_drift_kernel, dim3(nblk), dim3(256), 0, s, n, d, x, ldx, p, ldp, g,
                       inv_mass, step, mult, drift);
    return hipGetLastError();
}

// H = -(L - lambda/2 ||x||^2) + 1/2 sum p^2 / m  (one work-group, fixed order).
// Thread t adds elements t, t + T, ... (T = kEnergyThreads) in that order,
// loading kEnergyBatch of them per round so the loads are in flight together
// (an index past the end is clamped and its term dropped); each wave sums its
// lanes by DPP exchanges and thread 0 adds the waves in order.  Element
// indices are 32-bit: n D < 2^31 (the host bounds n through Y's leading
// dimension).
constexpr int kEnergyThreads = 1024;
constexpr int kEnergyBatch = 8;

__global__ void __launch_bounds__(kEnergyThreads)
    energy_kernel(int64_t n, int D, const double* x, int64_t ldx, const double* p, int64_t ldp,
                  const double* inv_mass, const double* prior, const double* loglik, double* out)
{
    __shared__ double s[2][kEnergyThreads / kWave];
    double kin = 0.0, pri = 0.0;
    const double lam = prior ? *prior : 0.0;
    const int ne = (int)(n * D);
    for (int e0 = threadIdx.x; e0 < ne; e0 += kEnergyBatch * kEnergyThreads) {
        double pv[kEnergyBatch], xv[kEnergyBatch], im[kEnergyBatch];
#pragma unroll
        for (int u = 0; u < kEnergyBatch; ++u) {
            const int e = min(e0 + u * kEnergyThreads, ne - 1);
            const int k = e / D, d = e - k * D;
            pv[u] = p[(int64_t)k * ldp + d];
            xv[u] = x[(int64_t)k * ldx + d];
            im[u] = inv_mass ? inv_mass[e] : 1.0;
        }
#pragma unroll
        for (int u = 0; u < kEnergyBatch; ++u) {
            if (e0 + u * kEnergyThreads < ne) {
                kin += 0.5 * pv[u] * pv[u] * im[u];
                pri += 0.5 * lam * xv[u] * xv[u];
            }
        }
    }
    kin = wave_sum(kin);
    pri = wave_sum(pri);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        s[0][w] = kin;
        s[1][w] = pri;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double k0 = 0.0, p0 = 0.0;
        for (int v = 0; v < kEnergyThreads / kWave; ++v) {
            k0 += s[0][v];
            p0 += s[1][v];
        }
        *out = -(*loglik - p0) + k0;
    }
}

hipError_t launch_energy(int64_t n, int d, const double* x, int64_t ldx, const double* p,
                         int64_t ldp, const double* inv_mass, const double* prior,
                         const double* loglik, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(energy_kernel, dim3(1), dim3(kEnergyThreads), 0, s, n, d, x, ldx, p, ldp,
                       inv_mass, prior, loglik, out);
    return hipGetLastError();
}

// ------------------------------------------------------------ prepare ---

__global__ void zero_i64_kernel(int64_t* p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// One work-group per row i: converts, folds the mask and NaN into NaN, and
// counts the observed pairs i > j of the row; one integer atomic per row
// (integer addition: the count does not depend on the order).
template <typename S, typename O>
__global__ void __launch_bounds__(256)
    prepare_kernel(const S* src, int64_t ld_src, const uint8_t* mask, int64_t ld_mask, O* out,
                   int64_t ldy, int64_t n, const int64_t* perm, unsigned long long* count)
{
    const int64_t i = blockIdx.x;
    O* orow = out + i * ldy;
    int obs = 0;
    if (perm) {
        // relabelled: out[i][j] = src[perm[i]][perm[j]]; an index out of
        // range reads as a missing pair
        const int64_t si = perm[i];
        const bool rok = si >= 0 && si < n;
        for (int64_t j = threadIdx.x; j < n; j += 256) {
            const int64_t sj = perm[j];
            bool miss = !(rok && sj >= 0 && sj < n);
            S v = (S)0;
            if (!miss) {
                v = src[si * ld_src + sj];
                miss = (mask && mask[si * ld_mask + sj] != 0) || isnan(v);
            }
            orow[j] = miss ? (O)NAN : (O)v;
            obs += (!miss && j < i) ? 1 : 0;
        }
    } else {
        const S* srow = src + i * ld_src;
        const uint8_t* mrow = mask ? mask + i * ld_mask : nullptr;
        for (int64_t j = threadIdx.x; j < n; j += 256) {
            const S v = srow[j];
            const bool miss = (mrow && mrow[j] != 0) || isnan(v);
            orow[j] = miss ? (O)NAN : (O)v;
            obs += (!miss && j < i) ? 1 : 0;
        }
    }
    if (count) {
        __shared__ int wsum[256 / kWave];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) obs += __shfl_xor(obs, m, kWave);
        if ((threadIdx.x & 63) == 0) wsum[threadIdx.x / kWave] = obs;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int q = 0; q < 256 / kWave; ++q) tot += wsum[q];
            if (tot) atomicAdd(count, (unsigned long long)tot);
        }
    }
}

hipError_t launch_prepare(const void* src, int sdt, int64_t ld_src, const uint8_t* mask,
                          int64_t ld_mask, void* out, int odt, int64_t ldy, int64_t n,
                          const int64_t* perm, int64_t* count, hipStream_t s)
{
    if (count) {
        hipLaunchKernelGGL(zero_i64_kernel, dim3(1), dim3(64), 0, s, count);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)n);
    unsigned long long* c = reinterpret_cast<unsigned long long*>(count);
    if (sdt == 0 && odt == 0)
        hipLaunchKernelGGL((prepare_kernel<double, double>), grid, dim3(256), 0, s,
                           (const double*)src, ld_src, mask, ld_mask, (double*)out, ldy, n, perm, c);
    else if (sdt == 0 && odt == 1)
        hipLaunchKernelGGL((prepare_kernel<double, float>), grid, dim3(256), 0, s,
                           (const double*)src, ld_src, mask, ld_mask, (float*)out, ldy, n, perm, c);
    else if (sdt == 1 && odt == 0)
        hipLaunchKernelGGL((prepare_kernel<float, double>), grid, dim3(256), 0, s,
                           (const float*)src, ld_src, mask, ld_mask, (double*)out, ldy, n, perm, c);
    else
        hipLaunchKernelGGL((prepare_kernel<float, float>), grid, dim3(256), 0, s,
                           (const float*)src, ld_src, mask, ld_mask, (float*)out, ldy, n, perm, c);
    return hipGetLastError();
}

// ---------------------------------------------------- symmetry check ---

// one work-group per row i: pairs (i, j < i) against (j, i); one integer
// atomic per row
template <typename T>
__global__ void __launch_bounds__(256)
    check_symmetric_kernel(const T* __restrict__ y, int64_t ldy, int64_t n,
                           unsigned long long* count)
{
    const int64_t i = blockIdx.x;
    int bad = 0;
    for (int64_t j = threadIdx.x; j < i; j += 256) {
        const T a = y[i * ldy + j], b = y[j * ldy + i];
        const bool same = (a == b) || (isnan(a) && isnan(b));
        bad += same ? 0 : 1;
    }
    __shared__ int wsum[256 / kWave];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) bad += __shfl_xor(bad, m, kWave);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x / kWave] = bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int q = 0; q < 256 / kWave; ++q) tot += wsum[q];
        if (tot) atomicAdd(count, (unsigned long long)tot);
    }
}

hipError_t launch_check_symmetric(const void* y, int dt, int64_t ldy, int64_t n, int64_t* count,
                                  hipStream_t s)
{
    hipLaunchKernelGGL(zero_i64_kernel, dim3(1), dim3(64), 0, s, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n == 0) return e;
    unsigned long long* c = reinterpret_cast<unsigned long long*>(count);
    if (dt == 0)
        hipLaunchKernelGGL((check_symmetric_kernel<double>), dim3((unsigned)n), dim3(256), 0, s,
                           (const double*)y, ldy, n, c);
    else
        hipLaunchKernelGGL((check_symmetric_kernel<float>), dim3((unsigned)n), dim3(256), 0, s,
                           (const float*)y, ldy, n, c);
    return hipGetLastError();
}

// ------------------------------------------------------ special funcs ---

__global__ void __launch_bounds__(256)
    log_phi_kernel(const double* t, double* lnphi, double* mills, int64_t count, int prec)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= count) return;
    double l, m;
    if (prec == 0) {
        log_phi_general_f64(t[e], l, m);
    } else {
        float lf, mf;
        log_phi_general_f32((float)t[e], lf, mf);
        l = lf;
        m = mf;
    }
    if (lnphi) lnphi[e] = l;
    if (mills) mills[e] = m;
}

hipError_t launch_log_phi(const double* t, double* lnphi, double* mills, int64_t count, int prec,
                          hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(log_phi_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, t,
                       lnphi, mills, count, prec);
    return hipGetLastError();
}

}  // namespace mds
