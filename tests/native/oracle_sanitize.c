/*
 * Drives every entry point of the C oracle on small problems -- empty, one
 * point, coincident points, masks, NaN (missing) entries, padded leading
 * dimensions -- so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer can catch an out-of-bounds access, a leak or
 * undefined arithmetic in it.  Inputs come from a small linear congruential
 * generator; nothing here computes the method.  Exit status 0 = every call
 * returned as documented and every output is finite.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_count_observed(int64_t n, const double* y, int64_t ldy, const unsigned char* mask,
                              int64_t ldm);
int oracle_eval(int64_t n, int d, const double* x, int64_t ldx, const double* y, int64_t ldy,
                const unsigned char* mask, int64_t ldm, double sigma, double* loglik,
                double* grad, double* dsigma, double* absrow, double* condrow, double* abs_l,
                double* abs_ds, int64_t* m_obs);
int oracle_eval_normal(int64_t n, int d, const double* x, int64_t ldx, const double* y,
                       int64_t ldy, const unsigned char* mask, int64_t ldm, double sigma,
                       double* loglik, double* grad, double* dsigma, double* absrow,
                       double* condrow, double* abs_l, double* abs_ds, int64_t* m_obs);
int oracle_lpd(int64_t n, int d, int64_t n_draws, const double* xs, const double* sigmas,
               const double* y, int64_t ldy, const unsigned char* mask, int64_t ldm,
               double* lpd, int64_t* m);
int oracle_leapfrog(int64_t n, int d, double* x, double* p, const double* y, int64_t ldy,
                    const unsigned char* mask, int64_t ldm, double sigma,
                    const double* inv_mass, double eps, double lambda, int n_steps,
                    double* grad_end, double* loglik_start, double* loglik_end,
                    double* energy_start, double* energy_end, int truncated);
int oracle_hmc_step(int64_t n, int d, double* x, const double* y, int64_t ldy,
                    const unsigned char* mask, int64_t ldm, double sigma,
                    const double* inv_mass, double eps, double lambda, int n_steps,
                    uint64_t seed, uint64_t it, double* p_out, double* grad_out,
                    double* loglik_out, double* h_start, double* h_end, double* log_u,
                    int* accepted, int truncated);
int oracle_grad_rows(int64_t n, int d, const double* x, int64_t ldx, const double* y,
                     int64_t ldy, const unsigned char* mask, int64_t ldm, double sigma,
                     const int64_t* rows, int64_t nrows, double* grad_rows, double* absrow,
                     double* condrow);
int oracle_grad_rows_given(int64_t n, int d, const double* x, int64_t ldx, const double* yrows,
                           int64_t ldyr, double sigma, const int64_t* rows, int64_t nrows,
                           double* grad_rows, double* absrow, double* condrow);

static uint64_t state = 12345u;
static double unif(void)
{
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

static int failures = 0;
static void check(int cond, const char* what, int64_t n, int d)
{
    if (!cond) {
        fprintf(stderr, "FAIL %s (n=%lld d=%d)\n", what, (long long)n, d);
        ++failures;
    }
}

static int all_finite(const double* v, int64_t k)
{
    for (int64_t i = 0; i < k; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* one problem: x (n x d, leading dimension ldx), symmetric y (ldy), mask */
static void run_case(int64_t n, int d, int coincident, double nan_frac, int use_mask)
{
    const int64_t ldx = d + 1, ldy = n + 3, ldm = n + 2;
    const size_t nx = (size_t)(n > 0 ? n : 1) * (size_t)ldx;
    const size_t ny = (size_t)(n > 0 ? n : 1) * (size_t)ldy;
    double* x = calloc(nx, sizeof(double));
    double* y = calloc(ny, sizeof(double));
    unsigned char* mask = calloc((size_t)(n > 0 ? n : 1) * (size_t)ldm, 1);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < d; ++k) x[i * ldx + k] = 3.0 * (unif() - 0.5);
    if (coincident && n >= 2)
        for (int k = 0; k < d; ++k) x[1 * ldx + k] = x[0 * ldx + k];
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < i; ++j) {
            double v = 0.05 + 2.0 * unif();
            if (unif() < nan_frac) v = NAN;
            y[i * ldy + j] = v;
            y[j * ldy + i] = v;
            const unsigned char mk = (unsigned char)(use_mask && unif() < 0.2);
            mask[i * ldm + j] = mk;
            mask[j * ldm + i] = mk;
        }
    }
    const unsigned char* mp = use_mask ? mask : NULL;
    const double sigma = 0.4;
    const int64_t nd = n * d;
    const size_t nb = (size_t)(nd > 0 ? nd : 1);

    const int64_t m = oracle_count_observed(n, y, ldy, mp, ldm);
    check(m >= 0 && m <= n * (n - 1) / 2, "count", n, d);

    double L, ds, absl, absds;
    int64_t mo = -1;
    double* g = calloc(nb, sizeof(double));
    double* ar = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double* cr = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    check(oracle_eval(n, d, x, ldx, y, ldy, mp, ldm, sigma, &L, g, &ds, ar, cr, &absl, &absds,
                      &mo) == 0,
          "eval", n, d);
    check(mo == m && isfinite(L) && isfinite(ds) && all_finite(g, nd), "eval outputs", n, d);
    check(oracle_eval_normal(n, d, x, ldx, y, ldy, mp, ldm, sigma, &L, g, &ds, ar, cr, &absl,
                             &absds, &mo) == 0 &&
              isfinite(L) && all_finite(g, nd),
          "eval_normal", n, d);
    /* only some outputs requested */
    check(oracle_eval(n, d, x, ldx, y, ldy, mp, ldm, sigma, &L, NULL, NULL, NULL, NULL, NULL,
                      NULL, NULL) == 0,
          "eval loglik only", n, d);

    if (n > 0) {
        int64_t rows[3] = {0, n - 1, n / 2};
        double gr[3 * 8], a3[3], b3[3];
        check(oracle_grad_rows(n, d, x, ldx, y, ldy, mp, ldm, sigma, rows, 3, gr, a3, b3) == 0 &&
                  all_finite(gr, 3 * d),
              "grad_rows", n, d);
        /* the listed rows whole, missing pairs as NaN */
        double* yr = calloc((size_t)(3 * n), sizeof(double));
        for (int r = 0; r < 3; ++r)
            for (int64_t j = 0; j < n; ++j) {
                const int64_t i = rows[r];
                yr[r * n + j] = (mp && mp[i * ldm + j]) ? NAN : y[i * ldy + j];
            }
        check(oracle_grad_rows_given(n, d, x, ldx, yr, n, sigma, rows, 3, gr, a3, b3) == 0 &&
                  all_finite(gr, 3 * d),
              "grad_rows_given", n, d);
        int64_t bad = n;
        check(oracle_grad_rows(n, d, x, ldx, y, ldy, mp, ldm, sigma, &bad, 1, gr, a3, b3) == -1,
              "grad_rows rejects a row out of range", n, d);
        free(yr);
    }

    /* leapfrog and HMC on contiguous x (ldx = d) */
    double* xc = calloc(nb, sizeof(double));
    double* p = calloc(nb, sizeof(double));
    double* im = calloc(nb, sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < d; ++k) {
            xc[i * d + k] = x[i * ldx + k];
            p[i * d + k] = unif() - 0.5;
            im[i * d + k] = 0.5 + unif();
        }
    for (int tr = 0; tr <= 1; ++tr) {
        double ge[64 * 8], l0, l1, e0, e1;
        double* gend = nd <= 64 * 8 ? ge : NULL;
        check(oracle_leapfrog(n, d, xc, p, y, ldy, mp, ldm, sigma, im, 1e-3, 0.1, 3, gend, &l0,
                              &l1, &e0, &e1, tr) == 0 &&
                  isfinite(l0) && isfinite(l1) && isfinite(e0) && isfinite(e1) &&
                  all_finite(xc, nd) && all_finite(p, nd),
              "leapfrog", n, d);
        double hs, he, lu;
        int acc = -1;
        check(oracle_hmc_step(n, d, xc, y, ldy, mp, ldm, sigma, NULL, 1e-3, 0.1, 2, 7u, 1u + tr,
                              p, g, &l1, &hs, &he, &lu, &acc, tr) == 0 &&
                  (acc == 0 || acc == 1) && all_finite(xc, nd),
              "hmc_step", n, d);
    }
    check(oracle_leapfrog(n, d, xc, p, y, ldy, mp, ldm, sigma, NULL, 1e-3, 0.0, -1, NULL, NULL,
                          NULL, NULL, NULL, 1) == -1,
          "leapfrog rejects negative steps", n, d);

    /* held-out density: the masked pairs held out, over three draws */
    if (n >= 2) {
        const int64_t S = 3;
        double* xs = calloc((size_t)(S * nd), sizeof(double));
        double sg[3] = {0.3, 0.4, 0.5};
        for (int64_t s = 0; s < S; ++s)
            for (int64_t k = 0; k < nd; ++k) xs[s * nd + k] = xc[k] + 0.01 * (double)s;
        double lpd;
        int64_t mh = -1;
        check(oracle_lpd(n, d, S, xs, sg, y, ldy, mp, ldm, &lpd, &mh) == 0 && mh >= 0 &&
                  isfinite(lpd),
              "lpd", n, d);
        free(xs);
    }
    free(x);
    free(y);
    free(mask);
    free(g);
    free(ar);
    free(cr);
    free(xc);
    free(p);
    free(im);
}

int main(void)
{
    const int64_t ns[] = {0, 1, 2, 7, 33};
    for (size_t a = 0; a < sizeof ns / sizeof ns[0]; ++a)
        for (int d = 1; d <= 8; d += 3) {
            run_case(ns[a], d, 0, 0.0, 0);
            run_case(ns[a], d, 1, 0.2, 1);
        }
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: ok\n");
    return 0;
}
