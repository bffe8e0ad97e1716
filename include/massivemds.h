/*
 * massivemds.h -- C-ABI of libmassivemds, the MI355X (gfx950) hot path of
 * Bayesian multidimensional scaling fitted by Hamiltonian Monte Carlo, after
 * Holbrook et al., "Massive parallelization boosts big Bayesian
 * multidimensional scaling" (arXiv:1905.04582).
 *
 * What it computes.  For N latent locations x_1..x_N in R^D (rows of X) and a
 * symmetric dissimilarity matrix Y, every unordered pair i > j contributes
 *     r_ij = (y_ij - delta_ij)^2 / (2 sigma^2) + ln Phi(delta_ij / sigma),
 *     delta_ij = ||x_i - x_j||_2,
 * and the log-likelihood of the truncated-normal observation model (Section
 * 2.1, Eq. 1 and Eq. 2) is
 *     L = -M ln sigma - sum_{observed i > j} r_ij,
 * with M the number of observed pairs and the 2*pi constant dropped (the
 * proportionality of Eq. 2).  The gradient rows are Eq. (9):
 *     dL/dx_i = -sum_{j != i} w_ij (x_i - x_j) / delta_ij,
 *     w_ij = (delta_ij - y_ij) / sigma^2 + phi(t) / (sigma Phi(t)), t = delta_ij/sigma,
 * and dL/dsigma = -M/sigma + sum [(y - delta)^2 / sigma^3 + delta phi(t)/(sigma^2 Phi(t))].
 * A coincident pair (delta = 0) contributes ln Phi(0) = -ln 2 to L and
 * nothing to the gradient.  With no observed pair, L = 0 and every
 * derivative is 0.
 *
 * Conventions shared by every entry point:
 *   - Every call returns an int status (MDS_OK or a negative MDS_ERR_*); the
 *     detail of the last failure on the calling thread is in mds_last_error().
 *     No C++ exception crosses this interface.
 *   - Arguments are validated on the host before any HIP call; a rejected
 *     call has no side effects.
 *   - Array arguments are DEVICE pointers owned by the caller; they must stay
 *     valid until the work enqueued on `stream` has completed.  Scalars that
 *     may change between replays of a captured graph (sigma, the step size,
 *     the upstream gradient scale, the prior precision) are device pointers
 *     to one double.
 *   - Every call is asynchronous on `stream` (NULL = the default stream),
 *     writes its results to device memory, never synchronises and never
 *     allocates: scratch memory is the caller's workspace, sized by
 *     mds_workspace_bytes().  Calls are therefore capturable into a HIP
 *     graph.  Calls that run concurrently need distinct workspaces.
 *   - X, the gradient, P and the mass diagonal are FP64.  Y is FP64
 *     (MDS_F64: FP64 pair arithmetic) or FP32 (MDS_F32: FP32 pair arithmetic
 *     with the pair difference formed and the sums finished in FP64).
 *   - Y is N x N row-major with leading dimension ldy >= N elements; only its
 *     strict lower triangle (row i > column j) is read, so Y must be
 *     symmetric for the result to be the paper's.  NaN entries are missing
 *     pairs (mds_prepare_y folds a mask into NaN).
 *   - sigma must be finite and > 0; this is not checked on the device (the
 *     value lives in device memory), a bad sigma yields NaN/Inf outputs.
 *     NaN or Inf in X or in observed entries of Y propagate to the outputs.
 *   - Results are deterministic: the same inputs on the same device give
 *     bitwise identical outputs (fixed-order reductions, no float atomics).
 *   - Pair tiling: `tile_rows` (rows per tile: 8, 16, 32, 64, 128 or 256) and
 *     `tile_waves` pick the tile shape and its waves; 0 selects the built-in
 *     default for (dtype, D, N).  tile_waves = MDS_TILE_WAVES(wc, wr): wc
 *     64-wide column groups per tile (1, 2, 4 or 8; the tile is 64*wc
 *     columns wide) and wr waves down the tile's rows (1, 2, 4 or 8; each
 *     walks tile_rows/wr >= 8 rows); wc * wr <= 8 waves per work-group.  A
 *     plain count (wr = 0 in the second byte) means wr = 1.  One of
 *     tile_rows and 64*wc must divide the other.  The workspace depends on
 *     tile_rows and wc only, and must be sized with the same values.
 */
#ifndef MASSIVEMDS_H
#define MASSIVEMDS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

/* The library is built with hidden visibility; these entry points are its
   only exported symbols. */
#define MDS_API __attribute__((visibility("default")))

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status -- */
enum mds_status {
    MDS_OK = 0,
    MDS_ERR_INVALID_ARGUMENT = -1, /* null pointer, bad size, bad stride, misalignment */
    MDS_ERR_UNSUPPORTED = -2,      /* D outside 1..MDS_MAX_DIM, unknown dtype, bad tiling */
    MDS_ERR_WORKSPACE_TOO_SMALL = -3,
    MDS_ERR_HIP = -4, /* a HIP runtime call failed; mds_last_error() names it */
    MDS_ERR_NOT_SYMMETRIC = -5 /* mds_require_symmetric found mismatched pairs */
};

/* element types */
enum mds_dtype { MDS_F64 = 0, MDS_F32 = 1 };

/* Model flag, OR-ed into the y_dtype argument of the evaluation calls
 * (mds_workspace_bytes, mds_resolve_tiling, mds_loglik, mds_gradient,
 * mds_leapfrog, mds_hmc_*, mds_batch_*): evaluate the model WITHOUT the
 * truncation to y > 0 -- plain normal errors, the ln Phi term of Eq. (2) and
 * the phi/Phi term of Eq. (9) left out -- the comparison the paper draws in
 * its scaling appendix. */
#define MDS_UNTRUNCATED 0x100

#define MDS_MAX_DIM 8
/* largest N accepted: tile and row indices are 32-bit on the device */
#define MDS_MAX_N ((int64_t)1 << 30)
/* workspace pointers must be aligned to this many bytes */
#define MDS_WORKSPACE_ALIGN 256
/* the tile_waves argument: wc column waves, wr row waves */
#define MDS_TILE_WAVES(wc, wr) ((int32_t)(wc) | ((int32_t)(wr) << 8))

/* Human-readable name of a status code (static string). */
MDS_API const char* mds_status_string(int status);

/* Detail of the last failed call on this thread ("" if none). */
MDS_API const char* mds_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
MDS_API int mds_version(void);

/*
 * Workspace size, in bytes, for mds_loglik / mds_gradient / mds_leapfrog on
 * an N-point, D-dimensional problem with the given Y dtype and tiling
 * (0 = default).  Writes *bytes; returns a status.
 */
MDS_API int mds_workspace_bytes(int64_t n, int32_t d, int32_t y_dtype, int32_t tile_rows,
                        int32_t tile_waves, size_t* bytes);

/*
 * The tiling the sweeps use for these arguments: tile_rows / tile_waves as
 * passed to mds_loglik and friends (0 = the library's default for n, d and
 * y_dtype), resolved and validated.  Writes *rows_out (rows per tile) and
 * *waves_out (the resolved MDS_TILE_WAVES(wc, wr); a plain count wc when
 * wr = 1);
 * returns a status (an unsupported tiling is MDS_ERR_UNSUPPORTED, as in the
 * evaluation calls).
 */
MDS_API int mds_resolve_tiling(int64_t n, int32_t d, int32_t y_dtype, int32_t tile_rows,
                       int32_t tile_waves, int32_t* rows_out, int32_t* waves_out);

/*
 * Prepare Y for the sweeps (not part of the per-evaluation path).
 *   y_src       N x N, dtype src_dtype, leading dimension ld_src (elements)
 *   missing     optional N x N bytes, leading dimension ld_mask; non-zero
 *               marks a missing pair (NULL = no mask).  Must be symmetric.
 *   y_out       N x N, dtype out_dtype, leading dimension ldy; receives
 *               y_src converted to out_dtype, with NaN where the mask is set
 *               or y_src is NaN.  y_out may alias y_src only when the two
 *               dtypes and leading dimensions are equal and perm is NULL.
 *   perm        optional device int64[N] (NULL = identity): relabel the
 *               locations, y_out[k][l] = y_src[perm[k]][perm[l]] (the mask
 *               likewise).  perm must be a permutation of 0..N-1; an entry
 *               outside that range makes its pairs missing.
 *   m_obs_dev   optional device int64: the number of observed pairs i > j.
 * Missing data are not part of the paper's model; they are excluded from
 * every sum and from M.
 */
MDS_API int mds_prepare_y(const void* y_src, int32_t src_dtype, int64_t ld_src,
                  const uint8_t* missing, int64_t ld_mask, void* y_out, int32_t out_dtype,
                  int64_t ldy, int64_t n, const int64_t* perm, int64_t* m_obs_dev,
                  hipStream_t stream);

/*
 * Symmetry check of a dissimilarity matrix (Eq. 1 defines y_ij for unordered
 * pairs; the sweeps read only the strict lower triangle, so an asymmetric Y
 * or mask silently gives the lower triangle's model).  Counts the pairs
 * i > j with y_ij != y_ji; two NaNs (two missing entries) count as equal, a
 * NaN against a number does not.  Checking a prepared Y therefore also checks
 * that the missing-pair mask was symmetric.
 *   y               N x N, dtype y_dtype, leading dimension ldy
 *   mismatches_dev  device int64 receiving the count (0 = symmetric)
 */
MDS_API int mds_check_symmetric(const void* y, int32_t y_dtype, int64_t ldy, int64_t n,
                        int64_t* mismatches_dev, hipStream_t stream);

/*
 * The checked mode of the symmetry test: mds_check_symmetric, then a wait for
 * `stream` and a read-back of the count.  Returns MDS_OK for a symmetric Y
 * and MDS_ERR_NOT_SYMMETRIC (mds_last_error() gives the count) otherwise.
 * Synchronous, so not capturable: a set-up call, once per prepared Y.
 * mismatches_dev is a caller-owned device int64 (it receives the count).
 */
MDS_API int mds_require_symmetric(const void* y, int32_t y_dtype, int64_t ldy, int64_t n,
                                  int64_t* mismatches_dev, hipStream_t stream);

/*
 * Spatial relabelling of the locations (a set-up step, not part of the
 * paper's method).  L of Eq. (2) sums over unordered pairs, so relabelling
 * the locations leaves L and dL/dsigma unchanged and permutes the gradient
 * rows of Eq. (9).  Under an order that keeps nearby locations at nearby
 * indices, the sweep skips the truncation terms of whole wavefronts whose
 * pairs all lie beyond its skip point, which makes every evaluation cheaper.
 *   x          N x D FP64 (ldx): the locations to order by (typically the
 *              starting X of a chain)
 *   perm       device int64[N] receiving the order: position k holds the
 *              original index of the k-th location along a Hilbert curve
 *              (D = 2) or in bit-interleaved (Morton) order (other D), over
 *              the bounding box of x quantised to 32-bit keys; ties keep
 *              index order.  Use it with mds_prepare_y(perm) for Y and
 *              mds_permute_rows for X, P and the gradient.
 *   workspace  device scratch of mds_order_workspace_bytes(n) bytes
 *              (MDS_WORKSPACE_ALIGN-aligned)
 */
MDS_API int mds_order_workspace_bytes(int64_t n, size_t* bytes);
MDS_API int mds_spatial_order(int64_t n, int32_t d, const double* x, int64_t ldx, int64_t* perm,
                      void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Relabel the rows of an N x D FP64 array by a permutation from
 * mds_spatial_order:
 *   inverse == 0: dst[k] = src[perm[k]]   (original labels -> relabelled)
 *   inverse != 0: dst[perm[k]] = src[k]   (relabelled -> original labels)
 * src and dst must not overlap.  An out-of-range perm entry writes a NaN row
 * (inverse == 0) or nothing (inverse != 0).
 */
MDS_API int mds_permute_rows(int64_t n, int32_t d, const double* src, int64_t ld_src, double* dst,
                     int64_t ld_dst, const int64_t* perm, int32_t inverse, hipStream_t stream);

/*
 * Log-likelihood L of Eq. (2) (see the header comment).
 *   x          N x D FP64, leading dimension ldx >= D
 *   y          prepared Y (y_dtype, ldy)
 *   sigma_dev  device double, sigma > 0
 *   loglik_dev device double receiving L
 */
MDS_API int mds_loglik(int64_t n, int32_t d, const double* x, int64_t ldx, const void* y,
               int32_t y_dtype, int64_t ldy, const double* sigma_dev, double* loglik_dev,
               void* workspace, size_t workspace_bytes, int32_t tile_rows, int32_t tile_waves,
               hipStream_t stream);

/*
 * Gradient of L with respect to X (Eq. 9), fused with L and dL/dsigma.
 *   scale_dev  optional device double s (NULL = 1): every output is
 *              multiplied by s (the upstream gradient of a reverse-mode
 *              caller: grad = s dL/dX, dsigma = s dL/dsigma; loglik is NOT
 *              scaled)
 *   grad       N x D FP64, leading dimension ldg >= D: s * dL/dX
 *   loglik_dev optional device double: L
 *   dsigma_dev optional device double: s * dL/dsigma
 *   dlogsigma_dev optional device double: s * dL/d(ln sigma) = s * sigma * dL/dsigma
 *              (the derivative a caller parametrising sigma by its log needs)
 */
MDS_API int mds_gradient(int64_t n, int32_t d, const double* x, int64_t ldx, const void* y,
                 int32_t y_dtype, int64_t ldy, const double* sigma_dev, const double* scale_dev,
                 double* grad, int64_t ldg, double* loglik_dev, double* dsigma_dev,
                 double* dlogsigma_dev, void* workspace, size_t workspace_bytes,
                 int32_t tile_rows, int32_t tile_waves, hipStream_t stream);

/*
 * mds_gradient for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same evaluation, outputs and arguments as mds_gradient, without a
 * workspace argument.  Its partial sums live in a static device array of
 * mds_noalloc_scratch_bytes() bytes (32 MiB) that the library holds on each
 * device for the life of the process; the call itself allocates nothing.
 * A problem whose workspace (mds_workspace_bytes with the same arguments)
 * exceeds that size is rejected with MDS_ERR_WORKSPACE_TOO_SMALL (at the
 * default tiling N = 5392 needs 11.2 MB in either dtype).  Every call on one
 * device shares that device's array: calls that overlap on one device (other
 * streams, other threads) race and must be ordered by the caller.  The first
 * call on a device looks the array's address up (hipGetSymbolAddress), which
 * is not capturable; make that first call outside a capture.
 */
MDS_API size_t mds_noalloc_scratch_bytes(void);
MDS_API int mds_gradient_noalloc(int64_t n, int32_t d, const double* x, int64_t ldx,
                                 const void* y, int32_t y_dtype, int64_t ldy,
                                 const double* sigma_dev, const double* scale_dev, double* grad,
                                 int64_t ldg, double* loglik_dev, double* dsigma_dev,
                                 double* dlogsigma_dev, int32_t tile_rows, int32_t tile_waves,
                                 hipStream_t stream);

/*
 * One leapfrog trajectory of Hamiltonian Monte Carlo (Section 2.3, Eqs. 6-8)
 * on the target log pi(X) = L(X) - (lambda/2) ||X||_F^2:
 *     p += (eps/2) grad log pi(x);
 *     n_steps - 1 times: x += eps M^{-1} p;  p += eps grad log pi(x);
 *     x += eps M^{-1} p;  p += (eps/2) grad log pi(x).
 *   x, p           N x D FP64 (leading dimensions ldx, ldp), updated in place
 *   inv_mass       optional N x D FP64 contiguous diagonal of M^{-1} (NULL = I)
 *   step_dev       device double eps
 *   prior_dev      optional device double lambda >= 0 (NULL = 0)
 *   n_steps        >= 0 (0: nothing moves, the outputs are still written)
 *   grad_io        N x D FP64 contiguous: grad log pi at x.  If cache_valid
 *                  is non-zero it must hold grad log pi(x) and loglik_io must
 *                  hold L(x) on entry, and the first gradient is not
 *                  recomputed.  On exit both describe the final x.
 *   loglik_io      device double: L (likelihood only, no prior) at x
 *   energy_start_dev, energy_end_dev
 *                  optional device doubles: H = -log pi(x) + p^T M^{-1} p / 2
 *                  (Eq. 6) before and after the trajectory
 * The workspace is the one of mds_gradient for the same (n, d, y_dtype, tiling).
 */
MDS_API int mds_leapfrog(int64_t n, int32_t d, double* x, int64_t ldx, double* p, int64_t ldp,
                 const void* y, int32_t y_dtype, int64_t ldy, const double* sigma_dev,
                 const double* inv_mass, const double* step_dev, const double* prior_dev,
                 int32_t n_steps, double* grad_io, double* loglik_io, int32_t cache_valid,
                 double* energy_start_dev, double* energy_end_dev, void* workspace,
                 size_t workspace_bytes, int32_t tile_rows, int32_t tile_waves,
                 hipStream_t stream);

/*
 * One Hamiltonian Monte Carlo transition (Section 2.3, Eqs. 6-8) of the
 * chain whose state is x, on the target log pi(X) = L(X) - (lambda/2)||X||^2
 * of mds_leapfrog: draw p ~ N(0, M), run one leapfrog trajectory of n_steps
 * steps, and accept the proposal with probability min(1, exp(H_start -
 * H_end)); a rejected proposal leaves x, grad_io and loglik_io as they were.
 *
 * Random draws (not part of the paper, which leaves them unspecified):
 * Philox4x32-10 (Salmon et al., SC 2011) with key (seed_lo, seed_hi) and
 * counter (k_lo, k_hi, it_lo, it_hi), where `it` = *iteration_dev is the
 * transition's index and k the draw's index; uniform(a, b) = ((a >> 6) 2^26
 * + (b >> 6) + 1/2) 2^-52 lies in (0, 1).  Momentum element e of the
 * row-major N x D array uses block k = e / 2: u1 = uniform(r0, r1), u2 =
 * uniform(r2, r3), z = sqrt(-2 ln u1) cos(2 pi u2) for even e and sin(2 pi
 * u2) for odd e, p_e = z / sqrt(inv_mass_e).  The test uses u = uniform(r0,
 * r1) of block k = 2^63 and accepts when ln u < H_start - H_end (never when
 * that difference is NaN).
 *
 *   x              N x D FP64 (ldx), the chain's state, updated in place
 *   iteration_dev  device uint64: the transition index; incremented by one
 *   p              N x D FP64 (ldp): the momentum at the trajectory's end
 *   grad_io, loglik_io, cache_valid
 *                  as in mds_leapfrog; on exit they describe the returned x
 *   stats_dev      optional device double[4]: H_start, H_end, ln u, accepted
 *                  (1.0 or 0.0)
 *   accepted_total_dev  optional device int64, incremented on acceptance
 *   workspace      mds_hmc_workspace_bytes() bytes (the gradient workspace
 *                  plus room to save the state)
 * Every step runs on the device and reads its scalars from device memory, so
 * transitions can be captured in a graph and replayed as a chain.
 */
MDS_API int mds_hmc_workspace_bytes(int64_t n, int32_t d, int32_t y_dtype, int32_t tile_rows,
                            int32_t tile_waves, size_t* bytes);
MDS_API int mds_hmc_step(int64_t n, int32_t d, double* x, int64_t ldx, const void* y, int32_t y_dtype,
                 int64_t ldy, const double* sigma_dev, const double* inv_mass,
                 const double* step_dev, const double* prior_dev, int32_t n_steps,
                 uint64_t seed, uint64_t* iteration_dev, double* p, int64_t ldp,
                 double* grad_io, double* loglik_io, int32_t cache_valid, double* stats_dev,
                 int64_t* accepted_total_dev, void* workspace, size_t workspace_bytes,
                 int32_t tile_rows, int32_t tile_waves, hipStream_t stream);

/*
 * The momentum draw of mds_hmc_step alone: p (N x D, ldp) = the momentum of
 * transition *iteration_dev under seed (iteration_dev is not incremented).
 */
MDS_API int mds_hmc_momentum(int64_t n, int32_t d, const double* inv_mass, uint64_t seed,
                     const uint64_t* iteration_dev, double* p, int64_t ldp, hipStream_t stream);

/*
 * Log pointwise predictive density of held-out pairs (the model-selection
 * part of Section 2): for each held-out pair, ln of the average over the
 * posterior draws s = 1..S of its truncated-normal density with the full
 * constant, ln p(y | delta, sigma) = -ln(sqrt(2 pi) sigma)
 * - (y - delta)^2 / (2 sigma^2) - ln Phi(delta / sigma); summed over pairs.
 *
 * 1. mds_heldout_count: the number of held-out pairs i > j (heldout byte
 *    non-zero, not missing: mask byte zero and y not NaN) into *m_dev, and
 *    the per-row offsets into the workspace (mds_heldout_workspace_bytes).
 * 2. mds_heldout_fill (same arguments and workspace): the pairs, in
 *    row-major order, into pi/pj (int32 row and column) and py (y as FP64);
 *    at most `capacity` are written.
 * 3. mds_lpd_accumulate, once per draw (x, sigma_dev): updates acc (2*m
 *    doubles, caller-owned: a running log-sum-exp per pair); first != 0
 *    starts it.  mds_lpd_accumulate_draws folds n_draws draws in one pass
 *    (draw s: x at xs + s * draw_stride doubles, leading dimension ldx,
 *    sigma = sigmas_dev[s]), in draw order, reading and writing acc once;
 *    the result is bit for bit that of n_draws single calls in the same
 *    order (first != 0 starts the sums with draw 0; n_draws = 0 does
 *    nothing).  The draws' arrays must not overlap acc.
 * 4. mds_lpd_finalize: lpd = sum over pairs of ln(average of the densities)
 *    over n_draws draws, into lpd_dev; its workspace (mds_lpd_workspace_bytes,
 *    256-byte aligned, caller-owned) holds partial sums.  The sums run in a
 *    fixed order, so the result is deterministic.
 */
MDS_API int mds_heldout_workspace_bytes(int64_t n, size_t* bytes);
MDS_API int mds_heldout_count(const void* y_src, int32_t src_dtype, int64_t ld_src,
                      const uint8_t* missing, int64_t ld_mask, const uint8_t* heldout,
                      int64_t ld_heldout, int64_t n, int64_t* m_dev, void* workspace,
                      size_t workspace_bytes, hipStream_t stream);
MDS_API int mds_heldout_fill(const void* y_src, int32_t src_dtype, int64_t ld_src,
                     const uint8_t* missing, int64_t ld_mask, const uint8_t* heldout,
                     int64_t ld_heldout, int64_t n, const void* workspace,
                     size_t workspace_bytes, int64_t capacity, int32_t* pi, int32_t* pj,
                     double* py, hipStream_t stream);
MDS_API int mds_lpd_accumulate(int64_t m, const int32_t* pi, const int32_t* pj, const double* py,
                       int32_t d, const double* x, int64_t ldx, const double* sigma_dev,
                       double* acc, int32_t first, hipStream_t stream);
MDS_API int mds_lpd_accumulate_draws(int64_t m, const int32_t* pi, const int32_t* pj,
                                     const double* py, int32_t d, const double* xs, int64_t ldx,
                                     int64_t draw_stride, const double* sigmas_dev,
                                     int32_t n_draws, double* acc, int32_t first,
                                     hipStream_t stream);
MDS_API int mds_lpd_workspace_bytes(int64_t m, size_t* bytes);
MDS_API int mds_lpd_finalize(int64_t m, const double* acc, int64_t n_draws, void* workspace,
                     size_t workspace_bytes, double* lpd_dev, hipStream_t stream);

/*
 * The device special functions of the sweeps, elementwise: ln Phi(t) and
 * phi(t)/Phi(t) (Eq. 2 and Eq. 9) for any real t, in the arithmetic of
 * `precision` (MDS_F64, or MDS_F32: t rounded to FP32 and FP32 arithmetic,
 * with the far lower tail t < -5 evaluated in FP64 by its log-erfc form).
 *   t, lnphi, mills   `count` FP64 values each (lnphi or mills may be NULL)
 */
MDS_API int mds_log_phi(const double* t, double* lnphi, double* mills, int64_t count,
                int32_t precision, hipStream_t stream);

/* ------------------------------------------------------------ batches -- */

/* One independent problem of a batch (every pointer a device pointer). */
typedef struct mds_problem_desc {
    int64_t n;             /* locations */
    int32_t d;             /* latent dimension, 1..MDS_MAX_DIM */
    int32_t tile_rows;     /* rows per tile (8/16/32/64/128/256); 0 = 128 rows, or the
                              single-problem default where 128 rows exceed the LDS budget */
    const double* x;       /* N x D FP64, leading dimension ldx (moved by mds_batch_leapfrog) */
    int64_t ldx;
    const void* y;         /* prepared Y, the batch's y_dtype, leading dimension ldy */
    int64_t ldy;
    const double* sigma;   /* device double, > 0 */
    const double* scale;   /* optional device double: multiplies grad, dsigma, dlogsigma */
    double* grad;          /* N x D FP64, leading dimension ldg (may be NULL for loglik only) */
    int64_t ldg;
    double* loglik;        /* optional device doubles */
    double* dsigma;
    double* dlogsigma;
    /* leapfrog (mds_batch_leapfrog only; NULL otherwise): momenta N x D FP64
       (leading dimension ldp, updated in place) and the step size eps as a
       device double */
    double* p;
    int64_t ldp;
    const double* step;
} mds_problem_desc;

/* What mds_batch_init leaves for mds_batch_eval: plain sizes and the
 * workspace it was initialised in.  Owned by the caller; no resources. */
typedef struct mds_batch_plan {
    int32_t count;
    int32_t y_dtype;
    int32_t tile_waves;      /* waves per work-group of the persistent sweep (wc * wr) */
    int32_t grid;            /* persistent work-groups */
    int32_t max_d;           /* largest D of the batch */
    int32_t flags;           /* bit 0: every problem has momenta, step, grad and loglik */
    int64_t total_tiles;
    int64_t elem_blocks;
    size_t lds_bytes;
    void* workspace;
    size_t workspace_bytes;
} mds_batch_plan;

/*
 * Many independent problems (uneven N, D) in one persistent sweep launch and
 * one finalize launch per evaluation.  Each problem's results equal, bit for
 * bit, those of mds_gradient with the same tile_rows and tile_waves.
 *   mds_batch_workspace_bytes: workspace for the batch (tile_waves common to
 *     the batch, 0 = MDS_TILE_WAVES(2, 1); y_dtype common to the batch; a
 *     descriptor's tile_rows 0 = 128 rows where the tiling allows, else the
 *     single-problem default).
 *   mds_batch_init: validates every descriptor, writes the device-side
 *     problem table into the workspace with one host-to-device copy on
 *     `stream` and waits for it (not capturable; call once per batch layout),
 *     and fills *plan.  The descriptors' pointers are baked into the table:
 *     later calls read and write those same buffers.
 *   mds_batch_eval: one evaluation of every problem (want_grad = 0: L only)
 *     on `stream`; asynchronous, allocation-free, capturable.  Calls sharing
 *     a workspace must not overlap.
 */
MDS_API int mds_batch_workspace_bytes(const mds_problem_desc* descs, int32_t count, int32_t y_dtype,
                              int32_t tile_waves, size_t* bytes);
MDS_API int mds_batch_init(const mds_problem_desc* descs, int32_t count, int32_t y_dtype,
                   int32_t tile_waves, void* workspace, size_t workspace_bytes,
                   mds_batch_plan* plan, hipStream_t stream);
MDS_API int mds_batch_eval(const mds_batch_plan* plan, int32_t want_grad, hipStream_t stream);

/*
 * Leapfrog trajectories (Section 2.3, Eqs. 6-8; unit mass, no prior) of
 * n_steps steps for every problem of the batch at once: each step is one
 * persistent batched sweep and one batched finalize that applies the kick
 * p += c eps grad and the drift x += eps p.  Every problem needs p, ldp >= d,
 * step, grad and loglik in its descriptor (plan->flags bit 0), else
 * MDS_ERR_INVALID_ARGUMENT.  x and p move in place; grad and loglik end at
 * the final x.  cache_valid != 0: grad holds grad L at the incoming x (the
 * previous trajectory's end) and the first evaluation is skipped.  Each
 * problem's x, p and gradient match mds_leapfrog on that problem alone with
 * the same tiling (unit mass, no prior), bit for bit.  Launches only: can be
 * captured in a graph.
 */
MDS_API int mds_batch_leapfrog(const mds_batch_plan* plan, int32_t n_steps, int32_t cache_valid,
                       hipStream_t stream);

/*
 * Diagnostics for benchmarks: while set (non-NULL), every single-problem
 * pair-sweep kernel launched by this thread records its own start in
 * `before` and its end in `after` (hipExtLaunchKernel), so a caller can time
 * the sweep kernel alone inside a larger sequence.  The events are the
 * caller's (created with timing enabled) and are recorded again by every
 * later sweep launch; pass NULL, NULL to stop.  Thread-local; no effect on
 * results.
 */
MDS_API int mds_set_sweep_events(hipEvent_t before, hipEvent_t after);

/*
 * Diagnostics for benchmarks: while `trace` is non-NULL, every single-problem
 * pair sweep launched by this thread writes, for wave w of the work-group of
 * tile t (in launch order), three uint64 at trace[(t * waves + w) * 3]: its
 * start and end reading of the 100 MHz real-time clock and its hardware slot
 * (the HW_ID register).  The caller sizes the buffer (ntiles * waves * 3
 * uint64, from mds_resolve_tiling); 8-byte aligned.  Thread-local; NULL
 * stops it; no effect on results.
 */
MDS_API int mds_set_tile_trace(void* trace);

#ifdef __cplusplus
}
#endif

#endif /* MASSIVEMDS_H */
