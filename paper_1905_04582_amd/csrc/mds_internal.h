// mds_internal.h -- tiling arithmetic and kernel launchers shared by the
// translation units of libmassivemds (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mds {

constexpr int kWave = 64;     // CDNA wavefront width

// Tile geometry of the lower-triangle pair sweep.
//
// Rows (index i) are cut into blocks of `br`, columns (index j) into blocks
// of `cw` = 64 * wc; one work-group owns one (row block, column block) tile.
// Its wc * wr waves form a grid: wave (u, v) owns the 64 consecutive columns
// u*64 .. u*64+63 of the tile and the v-th of wr equal groups of its rows, so
// wr > 1 shortens every wave's walk down the rows (and the time the last
// work-groups of a launch keep the machine partly idle) without changing the
// tile.  A tile exists when it can hold a pair with j < i.  With one of br
// and cw dividing the other, row block r holds a closed-form number of tiles,
// so a linear tile index maps back to (r, c) in closed form (tile_coords).
struct Tiling {
    int64_t n;
    int br;     // rows per tile
    int cw;     // columns per tile (64 * wc)
    int wc;     // waves across the tile's columns
    int wr;     // waves down the tile's rows (each walks br / wr rows)
    int waves;  // wc * wr: waves per work-group
    int nrb;    // number of row blocks
    int64_t ntiles;
    int elem;   // bytes of one Y element (8 in FP64, 4 in FP32): the staged rows' type
};

// br and cw are powers of two, so the ratios below are shifts
__host__ __device__ inline int log2_pow2(int v) { return __builtin_ctz((unsigned)v); }

__host__ __device__ inline int64_t tiles_in_row_block(int r, int br, int cw)
{
    if (br >= cw) return (int64_t)(r + 1) << (log2_pow2(br) - log2_pow2(cw));
    return (int64_t)(r >> (log2_pow2(cw) - log2_pow2(br))) + 1;
}

// number of tiles in row blocks 0..r-1
__host__ __device__ inline int64_t tiles_before(int r, int br, int cw)
{
    if (br >= cw) {
        const int sh = log2_pow2(br) - log2_pow2(cw);  // log2 of br / cw
        return (((int64_t)r * (r + 1)) >> 1) << sh;
    }
    const int sh = log2_pow2(cw) - log2_pow2(br);      // log2 of k = cw / br
    const int64_t a = r >> sh, b = r & ((1 << sh) - 1);
    return (int64_t)r + (((a * (a - 1)) >> 1) << sh) + a * b;
}

// first row block that holds a tile in column block c
__host__ __device__ inline int first_row_block_of_column(int c, int br, int cw)
{
    if (br >= cw) return c >> (log2_pow2(br) - log2_pow2(cw));
    return c << (log2_pow2(cw) - log2_pow2(br));
}

// (row block, column block) of linear tile index `tile` (row blocks in
// order, then column blocks in order within a row block), by a binary search
// on the prefix count (the reference form; the host tests compare the two)
__host__ __device__ inline void tile_coords_search(int64_t tile, int nrb, int br, int cw, int* r,
                                                   int* c)
{
    int lo = 0, hi = nrb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tiles_before(mid, br, cw) <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    *r = lo;
    *c = (int)(tile - tiles_before(lo, br, cw));
}

// The largest a >= 0 with a (a + 1) / 2 <= m, for 0 <= m < 2^31: the root
// of the triangular number in single precision (off by at most one), then
// corrected by one step either way in integers.
__host__ __device__ inline uint32_t tri_root(uint32_t m)
{
    uint32_t a = (uint32_t)((sqrtf(8.0f * (float)m + 1.0f) - 1.0f) * 0.5f);
    const uint64_t mm = m;
    if ((uint64_t)(a + 1) * (a + 2) / 2 <= mm) ++a;
    if (a > 0 && (uint64_t)a * (a + 1) / 2 > mm) --a;
    return a;
}

// tile_coords_search in closed form (32-bit: a tiling has fewer than 2^31
// tiles): with k = cw/br row blocks per column block, the a-th group of k row
// blocks holds k (a + 1) tiles; with k = br/cw column blocks per row block,
// row block r holds k (r + 1).  Either way the group is the root of a
// triangular number.  k is a power of two.
__host__ __device__ inline void tile_coords(int64_t tile, int nrb, int br, int cw, int* r, int* c)
{
    (void)nrb;
    const uint32_t g = (uint32_t)tile;
    const int lbr = __builtin_ctz((unsigned)br), lcw = __builtin_ctz((unsigned)cw);
    if (br <= cw) {
        const int sh = lcw - lbr;  // log2 k
        const uint32_t a = tri_root(g >> sh);
        // the group's first tile is k a (a + 1) / 2; its row blocks hold
        // a + 1 tiles each
        const uint32_t rem = g - ((a * (a + 1) / 2) << sh);
        const uint32_t b = rem / (a + 1);
        *r = (int)((a << sh) + b);
        *c = (int)(rem - b * (a + 1));
    } else {
        const int sh = lbr - lcw;
        const uint32_t a = tri_root(g >> sh);
        *r = (int)a;
        *c = (int)(g - ((a * (a + 1) / 2) << sh));
    }
}

// rows staged per reduction step of the sweep (keeps the per-wave staging
// buffer at <= 16 values per lane)
__host__ __device__ constexpr int sweep_stage_rows(int d) { return d <= 2 ? 8 : (d <= 4 ? 4 : 2); }

// The rows one wave of a tile walks.  The wave's row group is
// [rw0, rw1) (empty when the group lies past N); rows i <= jw0 hold no pair
// j < i for any of its lanes, so the walk starts at ib0, the last multiple
// of `rb` rows from rw0 at or below max(rw0, jw0 + 1).  The wave visits rows
// ib0 .. rw1-1 in order, and only when ib0 < rw1 (`active`); every row it
// reads -- its Y prefetch included -- lies in [ib0, rw1), inside both the
// tile and the matrix.
struct WaveRows {
    int row0, row1;  // the tile's rows [row0, row1), row1 <= n
    int rw0, rw1;    // the wave's row group, rw1 <= row1
    int jw0;         // the wave's first column
    int ib0;         // first row visited
    bool active;     // ib0 < rw1
};

// Row and column indices fit 32 bits (n <= 2^30 plus one tile); wc, wr and
// rb are powers of two, so the divisions are shifts.
__host__ __device__ inline WaveRows wave_rows(int64_t n, int br, int cw, int wc, int wr, int r,
                                              int c, int wave, int rb)
{
    WaveRows w;
    const int u = wave & (wc - 1), v = wave >> __builtin_ctz((unsigned)wc);
    const int rpw = br >> __builtin_ctz((unsigned)wr);
    const int n32 = (int)n;
    w.row0 = r * br;
    w.row1 = w.row0 + br < n32 ? w.row0 + br : n32;
    w.rw0 = w.row0 + v * rpw;
    const int e = w.rw0 + rpw;
    w.rw1 = e < w.row1 ? e : w.row1;
    w.jw0 = c * cw + u * 64;
    const int istart = w.rw0 > w.jw0 + 1 ? w.rw0 : w.jw0 + 1;
    w.ib0 = w.rw0 + (int)((unsigned)(istart - w.rw0) & ~(unsigned)(rb - 1));
    w.active = w.ib0 < w.rw1;
    return w;
}

inline Tiling make_tiling(int64_t n, int br, int wc, int wr, int elem)
{
    Tiling t;
    t.elem = elem;
    t.n = n;
    t.br = br;
    t.wc = wc;
    t.wr = wr;
    t.waves = wc * wr;
    t.cw = kWave * wc;
    t.nrb = (int)((n + br - 1) / br);
    t.ntiles = tiles_before(t.nrb, br, t.cw);
    return t;
}

// Workspace layout (each section aligned to 256 bytes).
struct WorkspaceLayout {
    size_t rowpart;  // ntiles * br * D doubles: row-side gradient partials
    size_t colpart;  // ncb * nrb * cw * D doubles: column-side gradient partials,
                     // slot (column block, row block); slots without a tile unused
    size_t tscal;    // ntiles * 2 doubles: per-tile sum r_ij and sum of dsigma terms
    size_t tcount;   // ntiles uint32: per-tile observed-pair count
    size_t total;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline WorkspaceLayout workspace_layout(const Tiling& t, int d)
{
    WorkspaceLayout w;
    size_t off = 0;
    w.rowpart = off;
    off = align_up(off + (size_t)t.ntiles * t.br * d * sizeof(double), 256);
    w.colpart = off;
    // column blocks that hold a tile: those of the last row block (with
    // br > cw this includes blocks past column n-1, whose tiles still write)
    const size_t ncb = t.nrb > 0 ? (size_t)tiles_in_row_block(t.nrb - 1, t.br, t.cw) : 0;
    off = align_up(off + ncb * (size_t)t.nrb * t.cw * d * sizeof(double), 256);
    w.tscal = off;
    off = align_up(off + (size_t)t.ntiles * 2 * sizeof(double), 256);
    w.tcount = off;
    off = align_up(off + (size_t)t.ntiles * sizeof(uint32_t), 256);
    w.total = off;
    return w;
}

// staged rows are padded by 32 bytes so that the rows a lane group reads in
// the transposed reduction start in different LDS banks
constexpr int kStagePadBytes = 32;

// LDS bytes used by one sweep work-group: tile row sums (one copy per
// column wave), per-wave scalars and the per-wave row staging buffer (rows of
// Y's element type, padded by kStagePadBytes; it also carries a wave's
// column sums when wr > 1, so it holds at least 64 * D doubles)
__host__ __device__ inline size_t sweep_stage_bytes(int d, int elem)
{
    const size_t rows = (size_t)sweep_stage_rows(d) * ((size_t)kWave * d * elem + kStagePadBytes);
    const size_t cols = (size_t)kWave * d * sizeof(double);
    return rows > cols ? rows : cols;
}

inline size_t sweep_lds_bytes(const Tiling& t, int d)
{
    return (size_t)t.wc * t.br * d * sizeof(double) + (size_t)t.waves * 4 * sizeof(double) +
           (size_t)t.waves * sweep_stage_bytes(d, t.elem);
}

// partial sums of the lpd finalize (its workspace holds this many doubles)
constexpr int kLpdMaxParts = 512;

struct SweepArgs {
    int64_t n;
    const double* x;
    int64_t ldx;
    const void* y;
    int64_t ldy;
    const double* sigma;
    int br, cw, nrb;
    int wc, wr;     // waves across columns and down rows of a tile
    double* rowpart;
    double* colpart;
    double* tscal;
    uint32_t* tcount;
    int truncated;  // 0: the model without the truncation terms (ln Phi = m = 0)
    // diagnostics (NULL in normal use): per wave of every tile, its start and
    // end clock (100 MHz) and hardware slot id
    unsigned long long* trace;
};

// What the finalize kernel does with the summed gradient of one element.
struct FinalizeArgs {
    int64_t n;
    int br, cw, nrb;
    int64_t ntiles;
    const double* rowpart;
    const double* colpart;
    const double* tscal;
    const uint32_t* tcount;
    const double* sigma;
    const double* scale;     // optional upstream scale (NULL = 1)
    double* grad;            // N x D output (ldg)
    int64_t ldg;
    double* loglik;          // optional
    double* dsigma;          // optional: scale * dL/dsigma
    double* dlogsigma;       // optional: scale * sigma * dL/dsigma
    // leapfrog extensions (all optional)
    const double* prior;     // lambda: grad -= lambda * x
    double* x;               // positions (ldx), drifted if drift != 0
    int64_t ldx;
    double* p;               // momenta (ldp), kicked if p != NULL
    int64_t ldp;
    const double* inv_mass;  // N x D contiguous diagonal of M^-1 (NULL = 1)
    const double* step;      // eps
    double kick_mult;        // kick coefficient = kick_mult * eps
    int drift;
};

// One problem of a batch, as the persistent kernels see it (device table).
struct BatchProblem {
    SweepArgs sweep;      // the problem's sweep arguments and partial buffers
    int32_t d;
    int32_t pad_;
    int64_t tile_base;    // global index of the problem's first tile
    int64_t ntiles;
    int64_t blk_base;     // first finalize element block of the problem
    int64_t nblk;         // finalize element blocks of the problem
    const double* scale;  // optional upstream scale
    double* grad;
    int64_t ldg;
    double* loglik;
    double* dsigma;
    double* dlogsigma;
    double* x;            // the problem's positions (drifted by the leapfrog)
    double* p;            // momenta (leapfrog only)
    int64_t ldp;
    const double* step;   // eps (leapfrog only)
};

// launchers (return hipError_t of the launch)
// start/stop (optional): events that record the sweep kernel's own start and
// end (hipExtLaunchKernel), for timing it alone
hipError_t launch_sweep(int y_dtype, int d, bool grad, const Tiling& t, const SweepArgs& a,
                        hipStream_t s, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
hipError_t launch_finalize(int d, const FinalizeArgs& a, hipStream_t s);
hipError_t launch_batch_sweep(int y_dtype, bool grad, int maxd, const BatchProblem* probs,
                              int32_t count, int64_t total_tiles, unsigned long long* cursor,
                              int waves, size_t lds, int grid, hipStream_t s);
int batch_sweep_blocks_per_cu(int y_dtype, bool grad, int maxd, int waves, size_t lds);
// kick_mult / kick / drift: the leapfrog update fused into the finalize
// (p += kick_mult eps g when kick, then x += eps p when drift); 0, 0, 0 for
// a plain evaluation
// blkmap: the problem of each finalize element block
hipError_t launch_batch_finalize(const BatchProblem* probs, const int32_t* blkmap, int32_t count,
                                 int64_t elem_blocks, unsigned long long* cursor, double kick_mult,
                                 int kick, int drift, hipStream_t s);
// p += kick_mult eps g, then x += eps p (drift != 0), every problem's elements
hipError_t launch_batch_kick_drift(const BatchProblem* probs, const int32_t* blkmap,
                                   int32_t count, int64_t elem_blocks, double kick_mult, int drift,
                                   hipStream_t s);

}  // namespace mds
