// mds_math.h -- device special functions of the truncated-normal MDS model.
//
// For t = delta/sigma >= 0 every pair needs ln Phi(t) (Eq. 2) and the ratio
// phi(t)/Phi(t) (Eq. 9).  Both are built branch-free from one exponential:
//     e = exp(-t^2/2),  z = t/sqrt 2,  erfcx(z) ~ P(z)/Q(z),
//     q = Phi(-t) = e erfcx(z) / 2 = a / (2Q)   with a = e P,
//     ln Phi(t) = log1p(-q) = -2 s A(s^2),  s = q/(2-q) = a / (4Q - a),
//     phi(t)/Phi(t) = e / (sqrt(2 pi) (1-q)) = 4 e Q / (sqrt(2 pi) (4Q - 2a)),
// where A(v) = atanh(sqrt v)/sqrt v.  s <= 1/3 because q <= 1/2, so A is a
// short polynomial on [0, 1/9], and log1p keeps full relative accuracy as
// q -> 0.  The two divisions share one reciprocal of (4Q - a)(4Q - 2a).
// Coefficients come from gen_coeffs.py (mds_coeffs.h).  Every lane runs the
// same instructions whatever t is: no branches, no lane divergence.
//
// The general helpers at the end also cover t < 0 (never reached by the
// sweeps, where delta >= 0 and sigma > 0) through the log-erfc form
//     ln Phi(t) = -t^2/2 + ln(erfcx(-t/sqrt 2)/2),
//     phi(t)/Phi(t) = sqrt(2/pi) / erfcx(-t/sqrt 2),
// which neither underflows nor cancels however far t goes below 0.
#pragma once

#include <hip/hip_runtime.h>

#include "mds_coeffs.h"

namespace mds {

constexpr double kInvSqrt2 = 0.70710678118654752440;
constexpr double kInvSqrt2Pi = 0.39894228040143267794;  // 1/sqrt(2 pi)
constexpr double kSqrt2OverPi = 0.79788456080286535588;  // sqrt(2/pi)

template <typename T, int N>
__device__ __forceinline__ T horner(const T (&c)[N], T x)
{
    T acc = c[N - 1];
#pragma unroll
    for (int k = N - 2; k >= 0; --k) acc = fma(acc, x, c[k]);
    return acc;
}

// acc * x + c with c in a scalar register: one VOP3 v_fma_f64.  (The
// compiler otherwise prefers the two-operand v_fmac_f64, whose addend must be
// a vector register, and copies every coefficient into one first.)
__device__ __forceinline__ double fma_sc(double acc, double x, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(acc), "v"(x), "s"(c));
    return r;
}

// The FP64 coefficient tables in one constant-memory object, so that one
// scalar base address reaches every coefficient by an immediate offset.
// terms of the series -log1p(-q)/q = sum_k q^k/(k+1) kept for q <= 1.5e-3
// (t >= 2.97): the next term is below 2e-18 of the sum
constexpr int kLog1pN = 6;

struct CoefTables64 {
    double exp[sizeof(kExpC64) / sizeof(double)];
    double erfcx_p[sizeof(kErfcxP64) / sizeof(double)];
    double erfcx_q[sizeof(kErfcxQ64) / sizeof(double)];
    double atanh[sizeof(kAtanhA64) / sizeof(double)];
    double erfcx_fp[sizeof(kErfcxFarP64) / sizeof(double)];
    double erfcx_fq[sizeof(kErfcxFarQ64) / sizeof(double)];
    double log1p[kLog1pN];  // 1/(k+1), k = 0 .. kLog1pN-1
};

constexpr CoefTables64 make_tables64()
{
    CoefTables64 t{};
    for (size_t k = 0; k < sizeof(kExpC64) / sizeof(double); ++k) t.exp[k] = kExpC64[k];
    for (size_t k = 0; k < sizeof(kErfcxP64) / sizeof(double); ++k) t.erfcx_p[k] = kErfcxP64[k];
    for (size_t k = 0; k < sizeof(kErfcxQ64) / sizeof(double); ++k) t.erfcx_q[k] = kErfcxQ64[k];
    for (size_t k = 0; k < sizeof(kAtanhA64) / sizeof(double); ++k) t.atanh[k] = kAtanhA64[k];
    for (size_t k = 0; k < sizeof(kErfcxFarP64) / sizeof(double); ++k)
        t.erfcx_fp[k] = kErfcxFarP64[k];
    for (size_t k = 0; k < sizeof(kErfcxFarQ64) / sizeof(double); ++k)
        t.erfcx_fq[k] = kErfcxFarQ64[k];
    for (int k = 0; k < kLog1pN; ++k) t.log1p[k] = 1.0 / (k + 1);
    return t;
}

static __constant__ CoefTables64 kTab64 = make_tables64();

typedef const __attribute__((address_space(4))) double* const_f64_ptr;
typedef const __attribute__((address_space(4))) CoefTables64* tab64_ptr;

// The tables' address, hidden from the optimiser by an empty asm: the
// coefficients are then fetched by uniform scalar loads (s_load) instead of
// being folded into immediates, which a 64-bit VALU operand cannot encode.
// A caller that evaluates the special functions in a loop takes the address
// once and passes it in.
__device__ __forceinline__ tab64_ptr tab64()
{
    tab64_ptr p = (tab64_ptr)&kTab64;
    asm volatile("" : "+s"(p));
    return p;
}

// Horner's rule over a table of N coefficients in constant memory.
template <int N>
__device__ __forceinline__ double horner_tab(const_f64_ptr c, double x)
{
    double acc = fma_sc(c[N - 1], x, c[N - 2]);
#pragma unroll
    for (int k = N - 3; k >= 0; --k) acc = fma_sc(acc, x, c[k]);
    return acc;
}

// Horner's rule for two arguments at once: each coefficient is loaded once
// and feeds both chains (two independent dependency chains interleave).
template <int N>
__device__ __forceinline__ void horner2_tab(const_f64_ptr c, double x1, double x2, double& r1,
                                            double& r2)
{
    double a1 = fma_sc(c[N - 1], x1, c[N - 2]);
    double a2 = fma_sc(c[N - 1], x2, c[N - 2]);
#pragma unroll
    for (int k = N - 3; k >= 0; --k) {
        a1 = fma_sc(a1, x1, c[k]);
        a2 = fma_sc(a2, x2, c[k]);
    }
    r1 = a1;
    r2 = a2;
}

// ---------------------------------------------------------------- FP64 --

// 1/d for finite d > 0 (not subnormal): hardware estimate + 2 Newton steps
__device__ __forceinline__ double rcp_f64(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// 1/sqrt(x) for finite x >= DBL_MIN: hardware estimate r (relative error
// below 2^-24 on gfx950), then one correction of third order: with
// e = (1 - x r^2)/2, 1/sqrt(x) = r (1 + e + 3/2 e^2 + 5/2 e^3 + ...), and
// the first omitted term is below 2^-70 of the result, so the final fma's
// rounding sets the error (a Newton step only squares it: two would be
// needed)
__device__ __forceinline__ double rsqrt_f64(double x)
{
    const double r = __builtin_amdgcn_rsq(x);
    const double e = fma(-0.5 * x, r * r, 0.5);
    return fma(r * e, fma(1.5, e, 1.0), r);
}

constexpr int kExpN = sizeof(kExpC64) / sizeof(double);
constexpr int kErfcxPN = sizeof(kErfcxP64) / sizeof(double);
constexpr int kErfcxQN = sizeof(kErfcxQ64) / sizeof(double);
constexpr int kAtanhN = sizeof(kAtanhA64) / sizeof(double);
constexpr int kErfcxFarPN = sizeof(kErfcxFarP64) / sizeof(double);
constexpr int kErfcxFarQN = sizeof(kErfcxFarQ64) / sizeof(double);

// exp(-t^2/2) for t >= 0; 0 once the value leaves the FP64 range
__device__ __forceinline__ double exp_neg_half_sq(double t, tab64_ptr tb)
{
    const double x = fmax(-0.5 * (t * t), -760.0);
    const double k = rint(x * kLog2e);
    double r = fma(k, -kLn2Head, x);
    r = fma(k, -kLn2Tail, r);
    return ldexp(horner_tab<kExpN>(tb->exp, r), (int)k);
}

// ln Phi(t) and phi(t)/Phi(t) for t >= 0 (the sweep's domain)
__device__ __forceinline__ void trunc_terms_f64(double t, double& lnphi, double& mills)
{
    const tab64_ptr tb = tab64();
    const double e = exp_neg_half_sq(t, tb);
    // beyond the fitted range e == 0, so any finite positive erfcx will do
    const double z = fmin(t * kInvSqrt2, kErfcxZmax64 + 1.0);
    const double P = horner_tab<kErfcxPN>(tb->erfcx_p, z);
    const double Q = horner_tab<kErfcxQN>(tb->erfcx_q, z);
    const double a = e * P;               // 2 q Q
    const double d1 = fma(4.0, Q, -a);    // 4Q - a   = 2Q (2 - q)
    const double d2 = d1 - a;             // 4Q - 2a  = 4Q (1 - q)
    const double rr = rcp_f64(d1 * d2);
    const double s = a * d2 * rr;         // q / (2 - q)
    lnphi = -2.0 * s * horner_tab<kAtanhN>(tb->atanh, s * s);
    mills = (4.0 * kInvSqrt2Pi) * (e * Q) * (d1 * rr);
}

// trunc_terms_f64 for two arguments, sharing every coefficient load; `tb`
// is the tables' address (tab64())
__device__ __forceinline__ void trunc_terms2_f64(double t1, double t2, double& lnphi1,
                                                 double& mills1, double& lnphi2, double& mills2,
                                                 tab64_ptr tb)
{
    const double x1 = fmax(-0.5 * (t1 * t1), -760.0);
    const double x2 = fmax(-0.5 * (t2 * t2), -760.0);
    const double k1 = rint(x1 * kLog2e), k2 = rint(x2 * kLog2e);
    double r1 = fma(k1, -kLn2Head, x1), r2 = fma(k2, -kLn2Head, x2);
    r1 = fma(k1, -kLn2Tail, r1);
    r2 = fma(k2, -kLn2Tail, r2);
    double p1, p2;
    horner2_tab<kExpN>(tb->exp, r1, r2, p1, p2);
    const double e1 = ldexp(p1, (int)k1), e2 = ldexp(p2, (int)k2);
    const double z1 = fmin(t1 * kInvSqrt2, kErfcxZmax64 + 1.0);
    const double z2 = fmin(t2 * kInvSqrt2, kErfcxZmax64 + 1.0);
    double P1, P2, Q1, Q2;
    horner2_tab<kErfcxPN>(tb->erfcx_p, z1, z2, P1, P2);
    horner2_tab<kErfcxQN>(tb->erfcx_q, z1, z2, Q1, Q2);
    const double a1 = e1 * P1, a2 = e2 * P2;
    const double d11 = fma(4.0, Q1, -a1), d12 = fma(4.0, Q2, -a2);
    const double d21 = d11 - a1, d22 = d12 - a2;
    const double rr1 = rcp_f64(d11 * d21), rr2 = rcp_f64(d12 * d22);
    const double s1 = a1 * d21 * rr1, s2 = a2 * d22 * rr2;
    double A1, A2;
    horner2_tab<kAtanhN>(tb->atanh, s1 * s1, s2 * s2, A1, A2);
    lnphi1 = -2.0 * s1 * A1;
    lnphi2 = -2.0 * s2 * A2;
    mills1 = (4.0 * kInvSqrt2Pi) * (e1 * Q1) * (d11 * rr1);
    mills2 = (4.0 * kInvSqrt2Pi) * (e2 * Q2) * (d12 * rr2);
}

// The same two pairs of values when both t lie at or past kFarT (up to the
// rounding of the caller's test, t >= 2.97): q = 1 - Phi(t) = exp(-t^2/2)
// erfcx(t/sqrt 2)/2 <= 1.5e-3 from the far-range rational, ln Phi = log1p(-q)
// by its series in q (kLog1pN terms), and phi/Phi = phi(t) / (1 - q) by the
// geometric series (terms to q^6, the next below 1.2e-17).  z is capped at
// the top of the fit range: past it exp(-t^2/2) < 1e-18, and the values are
// negligible however erfcx is approximated.
__device__ __forceinline__ void trunc_terms2_far_f64(double t1, double t2, double& lnphi1,
                                                     double& mills1, double& lnphi2,
                                                     double& mills2, tab64_ptr tb)
{
    const double x1 = fmax(-0.5 * (t1 * t1), -760.0);
    const double x2 = fmax(-0.5 * (t2 * t2), -760.0);
    const double k1 = rint(x1 * kLog2e), k2 = rint(x2 * kLog2e);
    double r1 = fma(k1, -kLn2Head, x1), r2 = fma(k2, -kLn2Head, x2);
    r1 = fma(k1, -kLn2Tail, r1);
    r2 = fma(k2, -kLn2Tail, r2);
    double p1, p2;
    horner2_tab<kExpN>(tb->exp, r1, r2, p1, p2);
    const double e1 = ldexp(p1, (int)k1), e2 = ldexp(p2, (int)k2);
    const double z1 = fmin(t1 * kInvSqrt2, kErfcxFarZmax64);
    const double z2 = fmin(t2 * kInvSqrt2, kErfcxFarZmax64);
    double P1, P2, Q1, Q2;
    horner2_tab<kErfcxFarPN>(tb->erfcx_fp, z1, z2, P1, P2);
    horner2_tab<kErfcxFarQN>(tb->erfcx_fq, z1, z2, Q1, Q2);
    const double q1 = 0.5 * (e1 * P1) * rcp_f64(Q1);
    const double q2 = 0.5 * (e2 * P2) * rcp_f64(Q2);
    double L1, L2;
    horner2_tab<kLog1pN>(tb->log1p, q1, q2, L1, L2);
    lnphi1 = -q1 * L1;
    lnphi2 = -q2 * L2;
    double g1 = 1.0, g2 = 1.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        g1 = fma(g1, q1, 1.0);
        g2 = fma(g2, q2, 1.0);
    }
    mills1 = kInvSqrt2Pi * e1 * g1;
    mills2 = kInvSqrt2Pi * e2 * g2;
}

// ---------------------------------------------------------------- FP32 --

// ln Phi(t) and phi(t)/Phi(t) for t >= 0 in FP32 arithmetic
__device__ __forceinline__ void trunc_terms_f32(float t, float& lnphi, float& mills)
{
    const float e = __builtin_amdgcn_exp2f(-0.5f * (t * t) * (float)kLog2e);
    const float z = fminf(t * (float)kInvSqrt2, kErfcxZmax32 + 1.0f);
    const float P = horner(kErfcxP32, z);
    const float Q = horner(kErfcxQ32, z);
    const float a = e * P;
    const float d1 = fmaf(4.0f, Q, -a);
    const float d2 = d1 - a;
    const float rr = __builtin_amdgcn_rcpf(d1 * d2);
    const float s = a * d2 * rr;
    lnphi = -2.0f * s * horner(kAtanhA32, s * s);
    mills = (float)(4.0 * kInvSqrt2Pi) * (e * Q) * (d1 * rr);
}

// --------------------------------------------------- general helpers ----

// any real t
__device__ inline void log_phi_general_f64(double t, double& lnphi, double& mills)
{
    if (t >= 0.0) {
        trunc_terms_f64(t, lnphi, mills);
    } else {
        // log-erfc form of the lower tail
        const double z = -t * kInvSqrt2;
        const double ex = erfcx(z);
        lnphi = -0.5 * t * t + log(0.5 * ex);
        mills = kSqrt2OverPi / ex;
    }
}

// any real t: FP32 arithmetic, except the far lower tail t < -5, which is
// evaluated in FP64 by the log-erfc form and rounded once.
__device__ inline void log_phi_general_f32(float t, float& lnphi, float& mills)
{
    if (t >= 0.0f) {
        trunc_terms_f32(t, lnphi, mills);
    } else if (t >= -5.0f) {
        const float z = -t * (float)kInvSqrt2;
        const float ex = erfcxf(z);
        lnphi = -0.5f * t * t + logf(0.5f * ex);
        mills = (float)kSqrt2OverPi / ex;
    } else {
        double l, m;
        log_phi_general_f64((double)t, l, m);
        lnphi = (float)l;
        mills = (float)m;
    }
}

}  // namespace mds
