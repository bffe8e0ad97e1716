// mds_order.hip -- spatial relabelling of the locations (a set-up step).
//
// L (Eq. 2) sums over unordered pairs and Eq. (9) gives one gradient row
// per location, so relabelling the locations by a permutation leaves L and
// dL/dsigma unchanged and permutes the gradient rows.  The sweep gains from
// a relabelling that puts nearby locations at nearby indices: the 64 columns
// of a wave then sit close together, and for most rows every one of them is
// far enough away that the wave skips the truncation terms.  The order used
// here is the Hilbert curve for D = 2 and bit interleaving (Morton order) for
// other D, on coordinates quantised over the bounding box of X.
//
// Everything runs in one work-group: a bounding-box pass, a key pass and a
// stable least-significant-digit radix sort (4-bit digits, 8 passes).  The
// cost is a few passes over N keys, once per problem.
#include "../../include/massivemds.h"
#include "mds_internal.h"

namespace mds {
namespace {

constexpr int kOrdThreads = 512;
constexpr int kOrdWaves = kOrdThreads / kWave;
constexpr int kDigitBits = 4;
constexpr int kDigits = 1 << kDigitBits;

// index of cell (qx, qy) along the Hilbert curve over a 2^b x 2^b grid
__device__ uint32_t hilbert_index(uint32_t qx, uint32_t qy, int b)
{
    const uint32_t full = (1u << b) - 1u;
    uint32_t h = 0;
    for (int k = b - 1; k >= 0; --k) {
        const uint32_t s = 1u << k;
        const uint32_t rx = (qx & s) ? 1u : 0u;
        const uint32_t ry = (qy & s) ? 1u : 0u;
        h += s * s * ((3u * rx) ^ ry);
        // reflect/transpose the lower bits into the sub-square's frame
        if (ry == 0) {
            if (rx) {
                qx ^= full;
                qy ^= full;
            }
            const uint32_t tmp = qx;
            qx = qy;
            qy = tmp;
        }
    }
    return h;
}

// bits per coordinate of the 32-bit key
__host__ __device__ inline int order_bits(int d) { return d == 1 ? 32 : (d == 2 ? 16 : 32 / d); }

// floor((v - lo) / (hi - lo) * (2^b - 1)); NaN and a flat box map to 0
__device__ uint32_t quantise(double v, double lo, double hi, int b)
{
    if (!(hi > lo)) return 0u;
    double t = (v - lo) / (hi - lo);
    if (!(t >= 0.0)) t = 0.0;
    if (t > 1.0) t = 1.0;
    const double top = (double)((b >= 32) ? 0xffffffffull : ((1ull << b) - 1ull));
    return (uint32_t)floor(t * top);
}

__device__ uint32_t point_key(const double* xi, int d, const double* lo, const double* hi)
{
    const int b = order_bits(d);
    if (d == 1) return quantise(xi[0], lo[0], hi[0], b);
    if (d == 2) return hilbert_index(quantise(xi[0], lo[0], hi[0], b),
                                     quantise(xi[1], lo[1], hi[1], b), b);
    uint32_t q[MDS_MAX_DIM];
    for (int dd = 0; dd < d; ++dd) q[dd] = quantise(xi[dd], lo[dd], hi[dd], b);
    uint32_t key = 0;
    for (int k = 0; k < b; ++k)
        for (int dd = 0; dd < d; ++dd) key |= ((q[dd] >> k) & 1u) << (k * d + dd);
    return key;
}

__global__ void __launch_bounds__(kOrdThreads)
    order_kernel(int64_t n, int d, const double* __restrict__ x, int64_t ldx, uint32_t* key0,
                 uint32_t* key1, uint32_t* idx0, uint32_t* idx1, int64_t* __restrict__ perm)
{
    __shared__ uint32_t hist[kDigits * kOrdThreads];  // [digit][thread]
    __shared__ double wlo[kOrdWaves][MDS_MAX_DIM], whi[kOrdWaves][MDS_MAX_DIM];
    __shared__ double lo[MDS_MAX_DIM], hi[MDS_MAX_DIM];
    __shared__ uint32_t wtot[kOrdWaves];
    const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;

    // bounding box (fmin/fmax skip NaN coordinates)
    for (int dd = 0; dd < d; ++dd) {
        double a = INFINITY, b = -INFINITY;
        for (int64_t i = t; i < n; i += kOrdThreads) {
            const double v = x[i * ldx + dd];
            a = fmin(a, v);
            b = fmax(b, v);
        }
        for (int m = 32; m >= 1; m >>= 1) {
            a = fmin(a, __shfl_xor(a, m, kWave));
            b = fmax(b, __shfl_xor(b, m, kWave));
        }
        if (lane == 0) {
            wlo[wv][dd] = a;
            whi[wv][dd] = b;
        }
    }
    __syncthreads();
    if (t < d) {
        double a = INFINITY, b = -INFINITY;
        for (int q = 0; q < kOrdWaves; ++q) {
            a = fmin(a, wlo[q][t]);
            b = fmax(b, whi[q][t]);
        }
        lo[t] = a;
        hi[t] = b;
    }
    __syncthreads();

    for (int64_t i = t; i < n; i += kOrdThreads) {
        key0[i] = point_key(x + i * ldx, d, lo, hi);
        idx0[i] = (uint32_t)i;
    }
    __syncthreads();

    // stable LSD radix sort: thread t owns the contiguous chunk [c0, c1)
    const int64_t chunk = (n + kOrdThreads - 1) / kOrdThreads;
    const int64_t c0 = min(n, (int64_t)t * chunk), c1 = min(n, c0 + chunk);
    uint32_t *ks = key0, *kd = key1, *is = idx0, *id = idx1;
    for (int shift = 0; shift < 32; shift += kDigitBits) {
        for (int g = 0; g < kDigits; ++g) hist[g * kOrdThreads + t] = 0u;
        for (int64_t i = c0; i < c1; ++i) ++hist[((ks[i] >> shift) & (kDigits - 1)) * kOrdThreads + t];
        __syncthreads();
        // exclusive scan of hist in (digit, thread) order: thread t scans the
        // kDigits consecutive entries starting at t * kDigits
        uint32_t* seg = hist + (size_t)t * kDigits;
        uint32_t local = 0;
        for (int k = 0; k < kDigits; ++k) local += seg[k];
        uint32_t inc = local;
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t u = __shfl_up(inc, o, kWave);
            if (lane >= o) inc += u;
        }
        if (lane == kWave - 1) wtot[wv] = inc;
        __syncthreads();
        uint32_t base = 0;
        for (int q = 0; q < wv; ++q) base += wtot[q];
        uint32_t run = base + inc - local;
        for (int k = 0; k < kDigits; ++k) {
            const uint32_t v = seg[k];
            seg[k] = run;
            run += v;
        }
        __syncthreads();
        for (int64_t i = c0; i < c1; ++i) {
            const uint32_t k = ks[i];
            const uint32_t pos = hist[((k >> shift) & (kDigits - 1)) * kOrdThreads + t]++;
            kd[pos] = k;
            id[pos] = is[i];
        }
        __syncthreads();
        uint32_t* tk = ks;
        ks = kd;
        kd = tk;
        uint32_t* ti = is;
        is = id;
        id = ti;
    }
    for (int64_t i = t; i < n; i += kOrdThreads) perm[i] = (int64_t)is[i];
}

__global__ void __launch_bounds__(256)
    permute_rows_kernel(int64_t n, int d, const double* __restrict__ src, int64_t ld_src,
                        double* __restrict__ dst, int64_t ld_dst, const int64_t* __restrict__ perm,
                        int inverse)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * d) return;
    const int64_t k = e / d;
    const int dd = (int)(e - k * d);
    const int64_t p = perm[k];
    const bool ok = p >= 0 && p < n;
    if (inverse) {
        if (ok) dst[p * ld_dst + dd] = src[k * ld_src + dd];
    } else {
        dst[k * ld_dst + dd] = ok ? src[p * ld_src + dd] : (double)NAN;
    }
}

}  // namespace

size_t order_workspace_bytes(int64_t n)
{
    const size_t one = align_up((size_t)n * sizeof(uint32_t), 256);
    return 4 * one;
}

hipError_t launch_order(int64_t n, int d, const double* x, int64_t ldx, int64_t* perm, void* ws,
                        hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const size_t one = align_up((size_t)n * sizeof(uint32_t), 256);
    char* base = static_cast<char*>(ws);
    uint32_t* k0 = reinterpret_cast<uint32_t*>(base);
    uint32_t* k1 = reinterpret_cast<uint32_t*>(base + one);
    uint32_t* i0 = reinterpret_cast<uint32_t*>(base + 2 * one);
    uint32_t* i1 = reinterpret_cast<uint32_t*>(base + 3 * one);
    hipLaunchKernelGGL(order_kernel, dim3(1), dim3(kOrdThreads), 0, s, n, d, x, ldx, k0, k1, i0,
                       i1, perm);
    return hipGetLastError();
}

hipError_t launch_permute_rows(int64_t n, int d, const double* src, int64_t ld_src, double* dst,
                               int64_t ld_dst, const int64_t* perm, int inverse, hipStream_t s)
{
    const int64_t total = n * d;
    if (total == 0) return hipSuccess;
    const dim3 grid((unsigned)((total + 255) / 256));
    hipLaunchKernelGGL(permute_rows_kernel, grid, dim3(256), 0, s, n, d, src, ld_src, dst, ld_dst,
                       perm, inverse);
    return hipGetLastError();
}

}  // namespace mds
