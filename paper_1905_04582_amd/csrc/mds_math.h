// mds_math.h -- device special functions of the truncated-normal MDS model.
//
// For t = delta/sigma >= 0 every pair needs ln Phi(t) (Eq. 2) and the ratio
// phi(t)/Phi(t) (Eq. 9).  Both come from q = Phi(-t) = erfc(t/sqrt 2)/2:
//     ln Phi(t) = log1p(-q)            (keeps relative accuracy as Phi -> 1)
//     phi(t)/Phi(t) = phi(t) / (1 - q)
// The general helpers below also cover t < 0 (not reached by the sweeps,
// where delta >= 0 and sigma > 0), through the scaled complementary error
// function: Phi(t) = exp(-t^2/2) erfcx(-t/sqrt 2) / 2, so
//     ln Phi(t) = -t^2/2 + ln(erfcx(-t/sqrt 2)/2),
//     phi(t)/Phi(t) = sqrt(2/pi) / erfcx(-t/sqrt 2),
// which neither underflows nor cancels however far t goes below 0.
#pragma once

#include <hip/hip_runtime.h>

namespace mds {

constexpr double kInvSqrt2 = 0.70710678118654752440;
constexpr double kInvSqrt2Pi = 0.39894228040143267794;  // 1/sqrt(2 pi)
constexpr double kSqrt2OverPi = 0.79788456080286535588;  // sqrt(2/pi)

// ---------------------------------------------------------------- FP64 --

// ln Phi(t) and phi(t)/Phi(t) for t >= 0 (the sweep's domain)
__device__ __forceinline__ void trunc_terms_f64(double t, double& lnphi, double& mills)
{
    const double q = 0.5 * erfc(t * kInvSqrt2);
    lnphi = log1p(-q);
    mills = (exp(-0.5 * t * t) * kInvSqrt2Pi) / (1.0 - q);
}

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

// ---------------------------------------------------------------- FP32 --

__device__ __forceinline__ void trunc_terms_f32(float t, float& lnphi, float& mills)
{
    const float q = 0.5f * erfcf(t * (float)kInvSqrt2);
    lnphi = log1pf(-q);
    mills = (expf(-0.5f * t * t) * (float)kInvSqrt2Pi) / (1.0f - q);
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
