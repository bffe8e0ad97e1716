/*
 * mds_oracle.c -- plain, serial, FP64 CPU oracle for the truncated-normal
 * multidimensional-scaling (MDS) likelihood of Holbrook et al.,
 * "Massive parallelization boosts big Bayesian multidimensional scaling".
 *
 * TEST INFRASTRUCTURE ONLY.  This file defines what the GPU path must
 * compute; it is slow on purpose (one pair at a time, compensated sums, libm
 * special functions) so that it can be checked against the paper by eye.
 * Only the test suite, the smoke check and the CPU-baseline leg of the bench
 * may load it.  It shares no code, header, table or constant with the HIP
 * library, and the HIP library never calls it.
 *
 * Conventions (the readings of the paper this oracle takes):
 *   - A pair (i, j) with i > j is one observation y_ij (Section 2.1, Eq. 1);
 *     each unordered pair is counted once.  Y is read from its lower triangle
 *     (row i, column j < i) of a row-major array with leading dimension ldy.
 *   - A pair is missing when its mask byte is non-zero or its y is NaN.
 *     Missing pairs are left out of the sums and of the count M.
 *   - The log-likelihood keeps the sigma normalisation of Eq. (2) for the
 *     observed pairs and drops the 2*pi constant, as the proportionality sign
 *     of Eq. (2) does:  L = -M ln(sigma) - sum_{observed i>j} r_ij,
 *     r_ij = (y_ij - delta_ij)^2 / (2 sigma^2) + ln Phi(delta_ij / sigma).
 *   - Gradient rows follow Eq. (9); a coincident pair (delta = 0) has an
 *     undefined direction and contributes zero to the gradient.
 *   - dL/dsigma is the derivative of the same L with respect to sigma.
 *   - Leapfrog follows Section 2.3 (Eqs. 6-8) with xdot = M^{-1} p (the
 *     printed factor 1/2 in Eq. 7 is read as a typesetting error) and an
 *     optional isotropic Gaussian prior -(lambda/2)||X||^2 in the target.
 *   - The HMC transition draws p ~ N(0, M) and the acceptance uniform from
 *     Philox4x32-10 (Salmon et al., SC 2011) counted by (draw, transition)
 *     and keyed by the seed; accept when ln u < H_start - H_end.
 *   - The model without truncation drops ln Phi from L and phi/Phi from the
 *     derivatives; the held-out predictive density averages the full
 *     truncated-normal density (with its 2 pi constant) over the draws.
 *
 * Every sum uses Neumaier's compensated summation, so the oracle's own
 * rounding error stays far below the 1e-12 parity tolerance even for tens of
 * millions of terms.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_SQRT2 1.41421356237309504880
#define ORACLE_LN_SQRT_2PI 0.91893853320467274178 /* ln(sqrt(2 pi)) */
#define ORACLE_INV_SQRT_2PI 0.39894228040143267794 /* 1/sqrt(2 pi) */

/* ---------------------------------------------------------------- sums -- */

typedef struct {
    double s; /* running sum */
    double c; /* running compensation */
} nsum;

static void nsum_add(nsum* a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double nsum_get(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------- normal distribution -- */

/* Mills ratio R(z) = Phi(-z)/phi(z) for z > 0 by Laplace's continued fraction
 * R(z) = 1/(z + 1/(z + 2/(z + 3/(z + ...)))), evaluated from the tail with a
 * fixed depth (used only for z >= 5, where 400 levels are far beyond
 * convergence in double precision). */
static double mills_ratio_cf(double z)
{
    double f = z;
    for (int k = 400; k >= 1; --k) f = z + (double)k / f;
    return 1.0 / f;
}

/* ln Phi(t), the log of the standard normal CDF named in Eq. (2), for any
 * real t.  For t >= 0 it is log1p(-Phi(-t)) with Phi(-t) = erfc(t/sqrt 2)/2,
 * which keeps full relative accuracy as Phi(t) -> 1.  For -5 <= t < 0 the
 * CDF itself is well conditioned.  Below -5 the Mills-ratio continued
 * fraction gives ln Phi(t) = ln phi(t) + ln R(-t) without underflow. */
double oracle_log_phi(double t)
{
    if (t >= 0.0) return log1p(-0.5 * erfc(t / ORACLE_SQRT2));
    if (t >= -5.0) return log(0.5 * erfc(-t / ORACLE_SQRT2));
    return -0.5 * t * t - ORACLE_LN_SQRT_2PI + log(mills_ratio_cf(-t));
}

/* phi(t)/Phi(t), the ratio that appears in the gradient of Eq. (9). */
double oracle_mills(double t)
{
    if (t >= -5.0) {
        double phi = exp(-0.5 * t * t) * ORACLE_INV_SQRT_2PI;
        return phi / (0.5 * erfc(-t / ORACLE_SQRT2));
    }
    return 1.0 / mills_ratio_cf(-t);
}

/* --------------------------------------------------------- likelihood -- */

static int pair_observed(int64_t i, int64_t j, const double* y, int64_t ldy,
                         const unsigned char* mask, int64_t ldm)
{
    if (mask && mask[i * ldm + j] != 0) return 0;
    return !isnan(y[i * ldy + j]);
}

/* Number of observed pairs i > j. */
int64_t oracle_count_observed(int64_t n, const double* y, int64_t ldy,
                              const unsigned char* mask, int64_t ldm)
{
    int64_t m = 0;
    for (int64_t i = 1; i < n; ++i)
        for (int64_t j = 0; j < i; ++j) m += pair_observed(i, j, y, ldy, mask, ldm);
    return m;
}

/*
 * Log-likelihood of Eq. (2), its gradient with respect to every row of X
 * (Eq. 9) and its derivative with respect to sigma, in one pass over the
 * pairs i > j.
 *
 *   x      n*d row-major, leading dimension ldx
 *   y      n*n row-major, leading dimension ldy (lower triangle read)
 *   mask   optional n*n bytes, leading dimension ldm; non-zero = missing
 *   sigma  observation standard deviation (> 0)
 * Outputs (each may be NULL):
 *   loglik    L
 *   grad      n*d row-major, contiguous: dL/dx_i
 *   dsigma    dL/dsigma
 *   absrow    n values: A_i = sum_j |w_ij|
 *   condrow   n values: B_i = sum_j [(delta_ij + |y_ij|)/sigma^2 + m_ij/sigma],
 *             the rounding scale of row i: w_ij = (delta - y)/sigma^2 + m/sigma
 *             subtracts two terms of size delta/sigma^2, so any 1-ulp change
 *             of delta moves w_ij by ~eps*delta/sigma^2 even when w_ij ~ 0
 *   abs_l     sum_j |r_ij| + M |ln sigma|, the scale of L's sum
 *   abs_ds    sum |dsigma terms| + M / sigma, the scale of dL/dsigma's sum
 *   m_obs     number of observed pairs
 * Returns 0, or -1 on bad arguments or allocation failure.
 *
 * With truncated = 0 the same pass evaluates the model without the
 * truncation to y > 0, i.e. plain normal errors y_ij ~ N(delta_ij, sigma^2)
 * (the comparison the paper draws in its scaling appendix): the ln Phi term
 * of Eq. (2) and the phi/Phi term of Eq. (9) are left out.
 */
static int eval_pairs(int64_t n, int d, const double* x, int64_t ldx, const double* y,
                      int64_t ldy, const unsigned char* mask, int64_t ldm, double sigma,
                      int truncated, double* loglik, double* grad, double* dsigma,
                      double* absrow, double* condrow, double* abs_l, double* abs_ds,
                      int64_t* m_obs)
{
    if (n < 0 || d < 1 || ldx < d || (n > 0 && ldy < n)) return -1;
    if (mask && n > 0 && ldm < n) return -1;

    nsum* g = NULL;
    nsum* a = NULL;
    nsum* b = NULL;
    if (n > 0) {
        g = (nsum*)calloc((size_t)(n * d), sizeof(nsum));
        a = (nsum*)calloc((size_t)n, sizeof(nsum));
        b = (nsum*)calloc((size_t)n, sizeof(nsum));
        if (!g || !a || !b) {
            free(g);
            free(a);
            free(b);
            return -1;
        }
    }
    nsum sr = {0, 0}, sr_abs = {0, 0}, ss = {0, 0}, ss_abs = {0, 0};
    int64_t m = 0;
    double* u = (double*)malloc(sizeof(double) * (size_t)d);
    if (!u) {
        free(g);
        free(a);
        free(b);
        return -1;
    }

    const double s2 = sigma * sigma;
    for (int64_t i = 1; i < n; ++i) {
        for (int64_t j = 0; j < i; ++j) {
            if (!pair_observed(i, j, y, ldy, mask, ldm)) continue;
            ++m;
            const double yij = y[i * ldy + j];
            /* delta_ij = ||x_i - x_j||_2  (Section 2.1) */
            double dd = 0.0;
            for (int k = 0; k < d; ++k) {
                double diff = x[i * ldx + k] - x[j * ldx + k];
                u[k] = diff;
                dd += diff * diff;
            }
            const double delta = sqrt(dd);
            const double t = delta / sigma;
            /* truncation terms of Eq. (2) and Eq. (9) */
            const double q = 0.5 * erfc(t / ORACLE_SQRT2); /* Phi(-t) */
            const double lnphi = truncated ? log1p(-q) : 0.0; /* ln Phi(t) */
            const double phi = exp(-0.5 * t * t) * ORACLE_INV_SQRT_2PI;
            const double mills = truncated ? phi / (1.0 - q) : 0.0; /* phi(t)/Phi(t) */
            const double resid = yij - delta;
            /* r_ij of Eq. (2) */
            const double r = resid * resid / (2.0 * s2) + lnphi;
            nsum_add(&sr, r);
            nsum_add(&sr_abs, fabs(r));
            /* the bracket of Eq. (9) */
            const double w = (delta - yij) / s2 + mills / sigma;
            nsum_add(&a[i], fabs(w));
            nsum_add(&a[j], fabs(w));
            const double cw = (delta + fabs(yij)) / s2 + mills / sigma;
            nsum_add(&b[i], cw);
            nsum_add(&b[j], cw);
            if (delta > 0.0) {
                for (int k = 0; k < d; ++k) {
                    const double c = w * (u[k] / delta);
                    nsum_add(&g[i * d + k], -c); /* row i: -w (x_i - x_j)/delta */
                    nsum_add(&g[j * d + k], c);  /* row j: the same pair, mirrored */
                }
            }
            /* d r_ij / d sigma, negated: contribution to dL/dsigma */
            const double ds = resid * resid / (s2 * sigma) + (delta / s2) * mills;
            nsum_add(&ss, ds);
            nsum_add(&ss_abs, fabs(ds));
        }
    }
    free(u);

    const double lns = log(sigma);
    if (loglik) {
        /* L = -M ln sigma - sum r: the sum is exact-compensated, the final
         * combination is one rounding */
        *loglik = -(double)m * lns - nsum_get(&sr);
        if (m == 0) *loglik = 0.0;
    }
    if (dsigma) *dsigma = (m == 0) ? 0.0 : -(double)m / sigma + nsum_get(&ss);
    if (abs_l) *abs_l = nsum_get(&sr_abs) + (double)m * fabs(lns);
    if (abs_ds) *abs_ds = nsum_get(&ss_abs) + (double)m / sigma;
    if (grad)
        for (int64_t k = 0; k < n * d; ++k) grad[k] = nsum_get(&g[k]);
    if (absrow)
        for (int64_t k = 0; k < n; ++k) absrow[k] = nsum_get(&a[k]);
    if (condrow)
        for (int64_t k = 0; k < n; ++k) condrow[k] = nsum_get(&b[k]);
    if (m_obs) *m_obs = m;
    free(g);
    free(a);
    free(b);
    return 0;
}

int oracle_eval(int64_t n, int d, const double* x, int64_t ldx, const double* y,
                int64_t ldy, const unsigned char* mask, int64_t ldm, double sigma,
                double* loglik, double* grad, double* dsigma, double* absrow,
                double* condrow, double* abs_l, double* abs_ds, int64_t* m_obs)
{
    return eval_pairs(n, d, x, ldx, y, ldy, mask, ldm, sigma, 1, loglik, grad, dsigma, absrow,
                      condrow, abs_l, abs_ds, m_obs);
}

/* The same outputs for the untruncated model (plain normal errors). */
int oracle_eval_normal(int64_t n, int d, const double* x, int64_t ldx, const double* y,
                       int64_t ldy, const unsigned char* mask, int64_t ldm, double sigma,
                       double* loglik, double* grad, double* dsigma, double* absrow,
                       double* condrow, double* abs_l, double* abs_ds, int64_t* m_obs)
{
    return eval_pairs(n, d, x, ldx, y, ldy, mask, ldm, sigma, 0, loglik, grad, dsigma, absrow,
                      condrow, abs_l, abs_ds, m_obs);
}

/*
 * Log pointwise predictive density of held-out pairs over posterior draws
 * (the model-selection subsection of Section 2: for each held-out pair, the
 * log of the Monte Carlo average over the S draws of the pair's predictive
 * density, summed over the held-out pairs).  The pair's density is the
 * truncated normal of Section 2.1 with its full normalising constant,
 *     ln p(y | delta, sigma) = -ln(sqrt(2 pi) sigma) - (y - delta)^2/(2 sigma^2)
 *                              - ln Phi(delta / sigma).
 *   xs      S draws of X, each n*d contiguous (row-major), one after another
 *   sigmas  S draws of sigma
 *   mask    every pair that is NOT held out (non-zero), as in oracle_eval
 * Writes the sum to *lpd and the number of held-out pairs to *m.  For S = 1
 * the value is the sum of the log densities at that one state.
 */
int oracle_lpd(int64_t n, int d, int64_t n_draws, const double* xs, const double* sigmas,
               const double* y, int64_t ldy, const unsigned char* mask, int64_t ldm,
               double* lpd, int64_t* m)
{
    if (n < 0 || d < 1 || n_draws < 1 || (n > 0 && ldy < n)) return -1;
    if (mask && n > 0 && ldm < n) return -1;
    double* l = (double*)malloc(sizeof(double) * (size_t)n_draws);
    if (!l) return -1;
    nsum total = {0, 0};
    int64_t cnt = 0;
    for (int64_t i = 1; i < n; ++i) {
        for (int64_t j = 0; j < i; ++j) {
            if (!pair_observed(i, j, y, ldy, mask, ldm)) continue;
            double lmax = -INFINITY;
            for (int64_t s = 0; s < n_draws; ++s) {
                const double* x = xs + s * n * d;
                const double sigma = sigmas[s];
                double dd = 0.0;
                for (int k = 0; k < d; ++k) {
                    const double diff = x[i * d + k] - x[j * d + k];
                    dd += diff * diff;
                }
                const double delta = sqrt(dd);
                const double z = (y[i * ldy + j] - delta) / sigma;
                const double log_norm = -ORACLE_LN_SQRT_2PI - log(sigma) - 0.5 * z * z;
                const double log_trunc = log1p(-0.5 * erfc(delta / sigma / ORACLE_SQRT2));
                l[s] = log_norm - log_trunc;
                if (l[s] > lmax) lmax = l[s];
            }
            /* log of the average of exp(l_s), shifted by the largest term */
            nsum acc = {0, 0};
            for (int64_t s = 0; s < n_draws; ++s) nsum_add(&acc, exp(l[s] - lmax));
            nsum_add(&total, lmax + log(nsum_get(&acc)) - log((double)n_draws));
            ++cnt;
        }
    }
    free(l);
    if (lpd) *lpd = nsum_get(&total);
    if (m) *m = cnt;
    return 0;
}

/* ----------------------------------------------------------- leapfrog -- */

/* gradient of the HMC target log pi(x) = L(x) - (lambda/2)||x||^2 */
static int target_grad(int64_t n, int d, const double* x, const double* y, int64_t ldy,
                       const unsigned char* mask, int64_t ldm, double sigma, double lambda,
                       int truncated, double* g, double* loglik)
{
    int rc = truncated ? oracle_eval(n, d, x, d, y, ldy, mask, ldm, sigma, loglik, g, NULL, NULL,
                                     NULL, NULL, NULL, NULL)
                       : oracle_eval_normal(n, d, x, d, y, ldy, mask, ldm, sigma, loglik, g, NULL,
                                            NULL, NULL, NULL, NULL, NULL);
    if (rc) return rc;
    if (lambda != 0.0)
        for (int64_t k = 0; k < n * d; ++k) g[k] -= lambda * x[k];
    return 0;
}

/*
 * One leapfrog trajectory of n_steps steps (Section 2.3).  x and p are n*d
 * contiguous and are updated in place.  inv_mass is an optional n*d diagonal
 * of M^{-1} (NULL = identity).  The momentum update uses p_dot = grad log pi
 * (Eq. 7): half kick, then n_steps-1 pairs of (drift, full kick), then a last
 * drift and half kick.
 *
 * Outputs (each may be NULL): grad_end = grad log pi at the final x,
 * loglik_start / loglik_end = L at the first and final x, and
 * energy_start / energy_end = H = -log pi(x) + p^T M^{-1} p / 2 (Eq. 6)
 * before and after the trajectory.  truncated = 0 targets the model without
 * the truncation to y > 0.
 */
int oracle_leapfrog(int64_t n, int d, double* x, double* p, const double* y, int64_t ldy,
                    const unsigned char* mask, int64_t ldm, double sigma,
                    const double* inv_mass, double eps, double lambda, int n_steps,
                    double* grad_end, double* loglik_start, double* loglik_end,
                    double* energy_start, double* energy_end, int truncated)
{
    if (n < 0 || d < 1 || n_steps < 0) return -1;
    const int64_t nd = n * d;
    double* g = (double*)malloc(sizeof(double) * (size_t)(nd > 0 ? nd : 1));
    if (!g) return -1;
    double L = 0.0;
    int rc = target_grad(n, d, x, y, ldy, mask, ldm, sigma, lambda, truncated, g, &L);
    if (rc) {
        free(g);
        return rc;
    }

    /* H = -log pi + kinetic, both as compensated sums */
    nsum kin = {0, 0}, pri = {0, 0};
    for (int64_t k = 0; k < nd; ++k) {
        const double im = inv_mass ? inv_mass[k] : 1.0;
        nsum_add(&kin, 0.5 * p[k] * p[k] * im);
        nsum_add(&pri, 0.5 * lambda * x[k] * x[k]);
    }
    if (loglik_start) *loglik_start = L;
    if (energy_start) *energy_start = -(L - nsum_get(&pri)) + nsum_get(&kin);

    if (n_steps > 0) {
        for (int64_t k = 0; k < nd; ++k) p[k] += 0.5 * eps * g[k];
        for (int s = 1; s <= n_steps; ++s) {
            for (int64_t k = 0; k < nd; ++k) x[k] += eps * (inv_mass ? inv_mass[k] : 1.0) * p[k];
            rc = target_grad(n, d, x, y, ldy, mask, ldm, sigma, lambda, truncated, g, &L);
            if (rc) {
                free(g);
                return rc;
            }
            const double c = (s < n_steps) ? eps : 0.5 * eps;
            for (int64_t k = 0; k < nd; ++k) p[k] += c * g[k];
        }
    }

    nsum kin2 = {0, 0}, pri2 = {0, 0};
    for (int64_t k = 0; k < nd; ++k) {
        const double im = inv_mass ? inv_mass[k] : 1.0;
        nsum_add(&kin2, 0.5 * p[k] * p[k] * im);
        nsum_add(&pri2, 0.5 * lambda * x[k] * x[k]);
    }
    if (loglik_end) *loglik_end = L;
    if (energy_end) *energy_end = -(L - nsum_get(&pri2)) + nsum_get(&kin2);
    if (grad_end) memcpy(grad_end, g, sizeof(double) * (size_t)nd);
    free(g);
    return 0;
}

/* ----------------------------------------------------- HMC transition -- */

/*
 * One Hamiltonian Monte Carlo transition (Section 2.3): draw the momentum
 * p ~ N(0, M), run one leapfrog trajectory, accept the proposal with
 * probability min(1, exp(H_start - H_end)) (Eq. 6 gives H), else keep x.
 *
 * The random draws come from the counter-based generator Philox4x32-10 of
 * Salmon, Moraes, Dror and Shaw ("Parallel random numbers: as easy as 1, 2,
 * 3", SC 2011): ten rounds of two 32x32->64-bit multiplications whose high
 * and low halves are mixed with the other counter words and the key, the key
 * advancing by the Weyl constants between rounds.  A block is indexed by a
 * 64-bit draw index k and the transition index `it`, keyed by the seed:
 *     block(k, it) = philox(counter = (k_lo, k_hi, it_lo, it_hi),
 *                           key = (seed_lo, seed_hi))
 * and a uniform in the open interval (0, 1) is made of 52 bits of two
 * output words (exact in FP64, so it never rounds to 0 or 1):
 *     uniform(a, b) = ((a >> 6) * 2^26 + (b >> 6) + 1/2) * 2^-52.
 * Momentum element e (row-major N x D) uses block k = e / 2 and the
 * Box-Muller transform: u1 = uniform(r0, r1), u2 = uniform(r2, r3),
 * z = sqrt(-2 ln u1) cos(2 pi u2) for even e, sin(2 pi u2) for odd e, and
 * p_e = z / sqrt(inv_mass_e) (variance M_e = 1 / inv_mass_e).  The
 * acceptance draw is u = uniform(r0, r1) of block k = 2^63; the proposal is
 * accepted when ln u < H_start - H_end (never when that is NaN).
 */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

double oracle_uniform_open(uint32_t a, uint32_t b)
{
    return ((double)(a >> 6) * 67108864.0 + (double)(b >> 6) + 0.5) / 4503599627370496.0;
}

static void draw_block(uint64_t k, uint64_t it, uint64_t seed, uint32_t r[4])
{
    const uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), (uint32_t)it, (uint32_t)(it >> 32)};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, r);
}

void oracle_momentum(int64_t n, int d, const double* inv_mass, uint64_t seed, uint64_t it,
                     double* p)
{
    const double two_pi = 6.28318530717958647692;
    for (int64_t e = 0; e < n * d; ++e) {
        uint32_t r[4];
        draw_block((uint64_t)(e / 2), it, seed, r);
        const double u1 = oracle_uniform_open(r[0], r[1]), u2 = oracle_uniform_open(r[2], r[3]);
        const double rad = sqrt(-2.0 * log(u1));
        const double z = (e % 2 == 0) ? rad * cos(two_pi * u2) : rad * sin(two_pi * u2);
        p[e] = z / sqrt(inv_mass ? inv_mass[e] : 1.0);
    }
}

double oracle_accept_uniform(uint64_t seed, uint64_t it)
{
    uint32_t r[4];
    draw_block((uint64_t)1 << 63, it, seed, r);
    return oracle_uniform_open(r[0], r[1]);
}

/*
 * x (n*d) is the chain's state, replaced by the proposal when it is
 * accepted.  p_out receives the momentum at the end of the trajectory,
 * grad_out and loglik_out grad log pi and L at the returned x.  h_start,
 * h_end, log_u and accepted report the Metropolis test.
 */
int oracle_hmc_step(int64_t n, int d, double* x, const double* y, int64_t ldy,
                    const unsigned char* mask, int64_t ldm, double sigma,
                    const double* inv_mass, double eps, double lambda, int n_steps,
                    uint64_t seed, uint64_t it, double* p_out, double* grad_out,
                    double* loglik_out, double* h_start, double* h_end, double* log_u,
                    int* accepted, int truncated)
{
    if (n < 0 || d < 1 || n_steps < 0 || !p_out || !grad_out) return -1;
    const int64_t nd = n * d;
    double* x0 = (double*)malloc(sizeof(double) * (size_t)(nd > 0 ? nd : 1));
    if (!x0) return -1;
    memcpy(x0, x, sizeof(double) * (size_t)nd);
    oracle_momentum(n, d, inv_mass, seed, it, p_out);
    double hs = 0.0, he = 0.0, L = 0.0;
    int rc = oracle_leapfrog(n, d, x, p_out, y, ldy, mask, ldm, sigma, inv_mass, eps, lambda,
                             n_steps, grad_out, NULL, &L, &hs, &he, truncated);
    if (rc) {
        free(x0);
        return rc;
    }
    const double lu = log(oracle_accept_uniform(seed, it));
    const int acc = lu < hs - he;
    if (!acc) {
        memcpy(x, x0, sizeof(double) * (size_t)nd);
        rc = target_grad(n, d, x, y, ldy, mask, ldm, sigma, lambda, truncated, grad_out, &L);
    }
    free(x0);
    if (loglik_out) *loglik_out = L;
    if (h_start) *h_start = hs;
    if (h_end) *h_end = he;
    if (log_u) *log_u = lu;
    if (accepted) *accepted = acc;
    return rc;
}

/* ------------------------------------------------------- sampled rows -- */

/*
 * Gradient rows of Eq. (9) for a subset of points only, for checks at sizes
 * where the full O(N^2) pass is too slow: for each listed row i, the sum over
 * every observed j != i of -w_ij (x_i - x_j)/delta_ij, with y_ij read from
 * the lower triangle (row max(i,j), column min(i,j)).  Also returns
 * A_i = sum_j |w_ij| and the rounding scale B_i of oracle_eval.  grad_rows
 * is nrows*d contiguous.
 */
/*
 * One gradient row of Eq. (9): point i against every j != i, where y_ij and
 * its mask byte are read as ylo[j] / mlo[j] for j < i and as
 * yhi[j * yst] / mhi[j * mst] for j > i (so the same code serves a row of
 * the lower triangle with its column, or a whole row of a symmetric
 * matrix).  u and g are caller scratch of d entries.
 */
static void grad_row(int64_t n, int d, const double* x, int64_t ldx, int64_t i,
                     const double* ylo, const double* yhi, int64_t yst,
                     const unsigned char* mlo, const unsigned char* mhi, int64_t mst,
                     double sigma, double* u, nsum* g, double* grad, double* absrow,
                     double* condrow)
{
    const double s2 = sigma * sigma;
    memset(g, 0, sizeof(nsum) * (size_t)d);
    nsum a = {0, 0}, b = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        const double yij = j < i ? ylo[j] : yhi[j * yst];
        const int missing = mlo ? (j < i ? mlo[j] : mhi[j * mst]) != 0 : 0;
        if (missing || isnan(yij)) continue;
        double dd = 0.0;
        for (int k = 0; k < d; ++k) {
            const double diff = x[i * ldx + k] - x[j * ldx + k];
            u[k] = diff;
            dd += diff * diff;
        }
        const double delta = sqrt(dd);
        const double t = delta / sigma;
        const double q = 0.5 * erfc(t / ORACLE_SQRT2);
        const double mills = exp(-0.5 * t * t) * ORACLE_INV_SQRT_2PI / (1.0 - q);
        const double w = (delta - yij) / s2 + mills / sigma;
        nsum_add(&a, fabs(w));
        nsum_add(&b, (delta + fabs(yij)) / s2 + mills / sigma);
        if (delta > 0.0)
            for (int k = 0; k < d; ++k) nsum_add(&g[k], -w * (u[k] / delta));
    }
    for (int k = 0; k < d; ++k) grad[k] = nsum_get(&g[k]);
    if (absrow) *absrow = nsum_get(&a);
    if (condrow) *condrow = nsum_get(&b);
}

int oracle_grad_rows(int64_t n, int d, const double* x, int64_t ldx, const double* y,
                     int64_t ldy, const unsigned char* mask, int64_t ldm, double sigma,
                     const int64_t* rows, int64_t nrows, double* grad_rows, double* absrow,
                     double* condrow)
{
    if (n < 0 || d < 1 || ldx < d || (n > 0 && ldy < n)) return -1;
    for (int64_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= n) return -1;
    double* u = (double*)malloc(sizeof(double) * (size_t)d);
    nsum* g = (nsum*)calloc((size_t)d, sizeof(nsum));
    if (!u || !g) {
        free(u);
        free(g);
        return -1;
    }
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows[r];
        grad_row(n, d, x, ldx, i, y + i * ldy, y + i, ldy, mask ? mask + i * ldm : NULL,
                 mask ? mask + i : NULL, ldm, sigma, u, g, grad_rows + r * d,
                 absrow ? absrow + r : NULL, condrow ? condrow + r : NULL);
    }
    free(u);
    free(g);
    return 0;
}

/*
 * The same for rows given whole: yrows holds, for each listed point i, row i
 * of the symmetric dissimilarity matrix (nrows x n, leading dimension ldyr;
 * y_ij = yrows[r][j], NaN = missing), so that rows can be checked at sizes
 * where Y itself does not fit host memory.
 */
int oracle_grad_rows_given(int64_t n, int d, const double* x, int64_t ldx, const double* yrows,
                           int64_t ldyr, double sigma, const int64_t* rows, int64_t nrows,
                           double* grad_rows, double* absrow, double* condrow)
{
    if (n < 0 || d < 1 || ldx < d || (nrows > 0 && ldyr < n)) return -1;
    for (int64_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= n) return -1;
    double* u = (double*)malloc(sizeof(double) * (size_t)d);
    nsum* g = (nsum*)calloc((size_t)d, sizeof(nsum));
    if (!u || !g) {
        free(u);
        free(g);
        return -1;
    }
    for (int64_t r = 0; r < nrows; ++r) {
        const double* yr = yrows + r * ldyr;
        grad_row(n, d, x, ldx, rows[r], yr, yr, 1, NULL, NULL, 0, sigma, u, g,
                 grad_rows + r * d, absrow ? absrow + r : NULL, condrow ? condrow + r : NULL);
    }
    free(u);
    free(g);
    return 0;
}
