// Host-only replay of the pair sweep's tile and wave arithmetic (no GPU).
//
// The sweep kernel maps a work-group index to a tile with tile_coords() (a
// closed form, checked against the prefix-count search tile_coords_search) and
// each of its waves to a row range with wave_rows(); this program calls the
// same functions (mds_internal.h) and checks, for many N, every valid tiling
// and the staging batch of every D:
//   * every row a wave reads -- its Y prefetch, which runs four rows ahead of
//     the arithmetic, and its x rows included -- lies inside its tile and
//     inside the matrix, and its staging batches cover its rows in order;
//   * the rows a wave skips below its first row hold no pair of its columns;
//   * every pair i > j of the strict lower triangle is visited exactly once
//     (counted pair by pair for small N, in total for large N);
//   * every partial-sum slot and LDS row a tile writes lies inside its
//     buffer, and the column-side slots of a column block are exactly those
//     the finalize reads (row blocks first_row_block_of_column(c) .. nrb-1).
// Exit status 0 and a summary line when every check holds; the first
// failure is printed with its case and the status is 1.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_1905_04582_amd/csrc/mds_internal.h"

using namespace mds;

static long long g_checks = 0;

#define CHECK(cond, ...)                                           \
    do {                                                           \
        ++g_checks;                                                \
        if (!(cond)) {                                             \
            std::fprintf(stderr, "FAIL %s:%d: %s -- ", __FILE__, __LINE__, #cond); \
            std::fprintf(stderr, __VA_ARGS__);                     \
            std::fprintf(stderr, "\n");                            \
            std::exit(1);                                          \
        }                                                          \
    } while (0)

struct Tile {
    int br, wc, wr;
};

// The rows the kernel's load_y() and next_x() read for one wave, and the
// first rows of the staging batches it closes.  The walk visits rows ib0,
// ib0+4, ... below rw1 in iterations of two steps of two rows (rows at or
// past rw1 are dead); Y is loaded four rows before the loop, then two rows
// after each step; x two rows per step.  Each pointer starts at ib0 and
// advances after a read while it is below the wave's last row.  A batch of
// rb rows closes after rb/2 steps, and a batch left open at the end closes
// after the loop.
static void replay_walk(const WaveRows& w, int rb, std::vector<int64_t>& yrows,
                        std::vector<int64_t>& xrows, std::vector<int64_t>& batches)
{
    yrows.clear();
    xrows.clear();
    batches.clear();
    if (!w.active) return;
    const int64_t last_row = w.rw1 - 1;
    int64_t ycur = w.ib0, ynext = w.ib0, xcur = w.ib0, xnext = w.ib0;
    auto load_y = [&]() {
        yrows.push_back(ycur);
        if (ynext < last_row) ++ycur;
        ++ynext;
    };
    auto next_x = [&]() {
        xrows.push_back(xcur);
        if (xnext < last_row) ++xcur;
        ++xnext;
    };
    for (int k = 0; k < 4; ++k) load_y();
    int q = 0;
    int64_t ib = w.ib0;
    for (; ib < w.rw1; ib += 4) {
        for (int half = 0; half < 2; ++half) {
            next_x();
            next_x();
            load_y();
            load_y();
            q += 2;
            if (q == rb) {
                batches.push_back(ib + 2 * (half + 1) - rb);
                q = 0;
            }
        }
    }
    if (q != 0) batches.push_back(ib - q);
}

// The fast walk (taken when the wave's rows are a whole number of
// iterations of max(rb, 4) rows and x rows are contiguous): Y rows ib0 ..
// ib0+3 first, then each iteration's four prefetched rows from one base row,
// capped at rw1-4 (the last iteration reads the wave's last four rows
// again); x rows ib0 .. rw1-1; a batch closed every rb rows.
static bool fast_walk(const WaveRows& w, int rb)
{
    const int it = rb > 4 ? rb : 4;
    return w.active && (w.rw1 - w.ib0) % it == 0;
}

// `misuse` counts steps whose register pair does not hold the Y rows the
// step evaluates.
static void replay_fast(const WaveRows& w, int rb, std::vector<int64_t>& yrows,
                        std::vector<int64_t>& xrows, std::vector<int64_t>& batches, int& misuse)
{
    yrows.clear();
    xrows.clear();
    batches.clear();
    misuse = 0;
    for (int k = 0; k < 4; ++k) yrows.push_back(w.ib0 + k);
    int64_t pa0 = w.ib0, pa1 = w.ib0 + 1, pb0 = w.ib0 + 2, pb1 = w.ib0 + 3;
    int64_t next = w.ib0 + 4;
    const int64_t cap = w.rw1 - 4;
    int q = 0;
    for (int64_t ib = w.ib0; ib < w.rw1; ib += 4) {
        const int64_t base = next < cap ? next : cap;
        next += 4;
        xrows.push_back(ib);
        xrows.push_back(ib + 1);
        misuse += (pa0 != ib || pa1 != ib + 1);
        pa0 = base;
        pa1 = base + 1;
        yrows.push_back(pa0);
        yrows.push_back(pa1);
        if (rb == 2) batches.push_back(ib);
        xrows.push_back(ib + 2);
        xrows.push_back(ib + 3);
        misuse += (pb0 != ib + 2 || pb1 != ib + 3);
        pb0 = base + 2;
        pb1 = base + 3;
        yrows.push_back(pb0);
        yrows.push_back(pb1);
        q += 4;
        if (q >= rb) {
            batches.push_back(ib + 4 - rb);
            q = 0;
        }
    }
}

// sum over k < m of min(max(k, 0), 64): the pairs of a wave's 64 columns in
// the rows i < jw0 + m
static long double pairs_below(int64_t m)
{
    if (m <= 1) return 0;
    const int64_t p = m - 1 < 64 ? m - 1 : 64;
    return (long double)(p * (p + 1) / 2) + 64.0L * (long double)(m - 65 > 0 ? m - 65 : 0);
}

static void check_case(int64_t n, const Tile& tl, int rb, bool per_pair, bool sample_tiles)
{
    const Tiling t = make_tiling(n, tl.br, tl.wc, tl.wr, 8);
    const int cw = t.cw;
    const int d = 1;
    const WorkspaceLayout lay = workspace_layout(t, d);
    const size_t rowpart_elems = (size_t)t.ntiles * t.br * d;
    const size_t colpart_elems = (lay.tscal - lay.colpart) / sizeof(double);
    const int64_t ncb = t.nrb > 0 ? tiles_in_row_block(t.nrb - 1, t.br, cw) : 0;
    std::vector<unsigned char> seen;
    if (per_pair) seen.assign((size_t)n * (size_t)n, 0);
    std::vector<int64_t> col_tiles(ncb > 0 ? ncb : 1, 0);
    std::vector<int64_t> loads, xloads, batches;
    long double pairs = 0;
    int64_t prev_tile_r = 0;
    for (int64_t tile = 0; tile < t.ntiles; ++tile) {
        int r, c, rs, cs;
        tile_coords(tile, t.nrb, t.br, cw, &r, &c);
        // the closed form the kernel uses against the prefix-count search
        tile_coords_search(tile, t.nrb, t.br, cw, &rs, &cs);
        CHECK(r == rs && c == cs, "n=%lld br=%d cw=%d tile=%lld: (%d,%d) vs (%d,%d)", (long long)n,
              t.br, cw, (long long)tile, r, c, rs, cs);
        CHECK(r >= 0 && r < t.nrb && c >= 0 && c < tiles_in_row_block(r, t.br, cw),
              "n=%lld br=%d cw=%d tile=%lld -> (%d,%d)", (long long)n, t.br, cw, (long long)tile, r, c);
        CHECK(tiles_before(r, t.br, cw) + c == tile && r >= prev_tile_r, "tile order n=%lld", (long long)n);
        prev_tile_r = r;
        CHECK(c < ncb, "column block %d >= %lld", c, (long long)ncb);
        CHECK(r >= first_row_block_of_column(c, t.br, cw), "tile (%d,%d) above its column's first row block", r, c);
        ++col_tiles[c];
        const bool full = !sample_tiles || r >= t.nrb - 3 || r == 0 || c + 1 == tiles_in_row_block(r, t.br, cw);
        // partial slots of the tile
        CHECK((size_t)(tile + 1) * t.br * d <= rowpart_elems, "rowpart of tile %lld", (long long)tile);
        CHECK((((size_t)c * t.nrb + r) * cw + cw) * d <= colpart_elems, "colpart slot (%d,%d)", c, r);
        if (!full) {
            // interior tiles far from the matrix edge: only the pair count
            // (row i holds min(max(i - jw0, 0), 64) pairs of the wave)
            for (int wv = 0; wv < t.waves; ++wv) {
                const WaveRows w = wave_rows(n, t.br, cw, t.wc, t.wr, r, c, wv, rb);
                if (w.active) pairs += pairs_below(w.rw1 - w.jw0) - pairs_below(w.ib0 - w.jw0);
            }
            continue;
        }
        for (int wv = 0; wv < t.waves; ++wv) {
            const WaveRows w = wave_rows(n, t.br, cw, t.wc, t.wr, r, c, wv, rb);
            const char* fmt = "n=%lld br=%d wc=%d wr=%d rb=%d tile=(%d,%d) wave=%d";
#define CASE (long long)n, t.br, t.wc, t.wr, rb, r, c, wv
            CHECK(w.row0 == (int64_t)r * t.br && w.row0 < n && w.row1 <= n && w.row1 > w.row0, fmt, CASE);
            CHECK(w.rw0 >= w.row0 && w.rw1 <= w.row1, fmt, CASE);
            CHECK(w.jw0 == (int64_t)c * cw + (int64_t)(wv % t.wc) * 64, fmt, CASE);
            // LDS rows the wave zeroes and writes: inside the tile's br rows
            if (w.rw1 > w.rw0) CHECK(w.rw1 - w.row0 <= t.br, fmt, CASE);
            // rows skipped below the first visited row hold no pair
            for (int64_t i = w.rw0; i < w.ib0 && i < w.rw1; ++i) CHECK(i <= w.jw0, fmt, CASE);
            if (!w.active) {
                // an inactive wave's rows hold no pair either
                for (int64_t i = w.rw0; i < w.rw1; ++i) CHECK(i <= w.jw0, fmt, CASE);
                continue;
            }
            CHECK((w.ib0 - w.rw0) % rb == 0 && w.ib0 >= w.rw0, fmt, CASE);
            replay_walk(w, rb, loads, xloads, batches);
            for (int64_t y : loads) {
                CHECK(y >= w.ib0 && y < w.rw1, "%s load row %lld", "", (long long)y);
                CHECK(y >= w.row0 && y < w.row1 && y < n, fmt, CASE);
            }
            for (int64_t x : xloads) CHECK(x >= w.ib0 && x < w.rw1 && x < n, fmt, CASE);
            // the staging batches: consecutive runs of rb rows from ib0 that
            // cover [ib0, rw1); the row sums a batch writes (its live rows)
            // lie in the wave's rows of the tile
            CHECK(!batches.empty() && batches.front() == w.ib0, fmt, CASE);
            // (a batch that starts at or past rw1 has only dead rows and
            // writes nothing)
            int64_t live_batches = 0;
            for (size_t b = 0; b < batches.size(); ++b) {
                CHECK(batches[b] == w.ib0 + (int64_t)b * rb, fmt, CASE);
                CHECK(batches[b] >= w.row0, fmt, CASE);
                if (batches[b] < w.rw1) ++live_batches;
            }
            CHECK(live_batches * rb >= w.rw1 - w.ib0 && (live_batches - 1) * rb < w.rw1 - w.ib0,
                  fmt, CASE);
            if (fast_walk(w, rb)) {
                // the fast walk: every Y and x row it reads lies in the
                // wave's rows; batches cover the rows exactly, in order
                int misuse = 0;
                replay_fast(w, rb, loads, xloads, batches, misuse);
                CHECK(misuse == 0, fmt, CASE);
                for (int64_t y : loads) CHECK(y >= w.ib0 && y < w.rw1 && y < n, fmt, CASE);
                for (int64_t x : xloads) CHECK(x >= w.ib0 && x < w.rw1, fmt, CASE);
                CHECK((int64_t)batches.size() * rb == w.rw1 - w.ib0, fmt, CASE);
                for (size_t b = 0; b < batches.size(); ++b)
                    CHECK(batches[b] == w.ib0 + (int64_t)b * rb, fmt, CASE);
            }
            if (!per_pair) {
                pairs += pairs_below(w.rw1 - w.jw0) - pairs_below(w.ib0 - w.jw0);
                continue;
            }
            for (int64_t i = w.ib0; i < w.rw1; ++i) {
                for (int l = 0; l < 64; ++l) {
                    const int64_t j = w.jw0 + l;
                    if (j >= n || j >= i) continue;
                    pairs += 1;
                    if (per_pair) {
                        unsigned char& s = seen[(size_t)i * n + j];
                        CHECK(s == 0, "pair (%lld,%lld) twice: n=%lld br=%d wc=%d wr=%d", (long long)i,
                              (long long)j, (long long)n, t.br, t.wc, t.wr);
                        s = 1;
                    }
                }
            }
#undef CASE
        }
    }
    // the finalize's row-side lists: row block r's tiles are the run
    // tiles_before(r) .. + tiles_in_row_block(r)
    for (int r = 0; r < t.nrb; ++r)
        CHECK(tiles_before(r + 1, t.br, cw) == tiles_before(r, t.br, cw) + tiles_in_row_block(r, t.br, cw),
              "row block %d of n=%lld br=%d cw=%d", r, (long long)n, t.br, cw);
    CHECK(tiles_before(t.nrb, t.br, cw) == t.ntiles, "tile count n=%lld", (long long)n);
    // column-side slots: one tile in each row block from the first of the column
    for (int64_t c = 0; c < ncb; ++c)
        CHECK(col_tiles[c] == t.nrb - first_row_block_of_column((int)c, t.br, cw),
              "column block %lld has %lld tiles", (long long)c, (long long)col_tiles[c]);
    const long double want = (long double)n * (long double)(n - 1) / 2;
    CHECK(pairs == want, "n=%lld br=%d wc=%d wr=%d rb=%d: %.0Lf pairs visited, %.0Lf in the triangle",
          (long long)n, t.br, t.wc, t.wr, rb, pairs, want);
    if (per_pair)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < i; ++j)
                CHECK(seen[(size_t)i * n + j] == 1, "pair (%lld,%lld) not visited", (long long)i, (long long)j);
}

int main()
{
    std::vector<Tile> tilings;
    const int rows[] = {8, 16, 32, 64, 128, 256};
    const int cnts[] = {1, 2, 4, 8};
    for (int br : rows)
        for (int wc : cnts)
            for (int wr : cnts) {
                const int cw = 64 * wc;
                if (wc * wr > 8 || br / wr < 8 || !(br % cw == 0 || cw % br == 0)) continue;
                tilings.push_back({br, wc, wr});
            }
    std::vector<int64_t> ns;
    for (int64_t n = 1; n <= 600; ++n) ns.push_back(n);
    for (int64_t n : {777, 1000, 1536, 5000, 5392, 7999, 20000, 100000}) ns.push_back(n);
    const int rbs[] = {sweep_stage_rows(1), sweep_stage_rows(3), sweep_stage_rows(6)};
    long long cases = 0;
    for (int64_t n : ns)
        for (const Tile& tl : tilings)
            for (int rb : rbs) {
                // the largest problems: tiles of 32 rows or more, and the
                // extreme staging batches
                if (n >= 20000 && (tl.br < 32 || rb == sweep_stage_rows(3))) continue;
                const bool per_pair = n <= 96 || n == 257 || n == 600 || n == 1000;
                const bool sample = n >= 5000;
                check_case(n, tl, rb, per_pair, sample);
                ++cases;
            }
    std::printf("tile bounds ok: %lld cases (%zu tilings), %lld checks\n", cases, tilings.size(),
                g_checks);
    return 0;
}
