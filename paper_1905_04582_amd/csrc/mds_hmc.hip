// mds_hmc.hip -- the device kernels of one HMC transition (Section 2.3)
// around the leapfrog trajectory: momentum draw and state save, the
// Metropolis test, and the restore of a rejected proposal.  All state
// (the transition counter, the energies, the decision) stays in device
// memory, so a transition or a chain of them can be captured in a graph.
#include "mds_internal.h"
#include "mds_rng.h"

namespace mds {
namespace {

// p = momentum of transition *iteration (N x D, ldp); optionally save x,
// grad and L for a possible rejection
__global__ void __launch_bounds__(256)
    hmc_begin_kernel(int64_t n, int d, const double* __restrict__ inv_mass, uint64_t seed,
                     const uint64_t* __restrict__ iteration, double* __restrict__ p, int64_t ldp,
                     const double* __restrict__ x, int64_t ldx, const double* __restrict__ grad,
                     const double* __restrict__ loglik, double* __restrict__ x_save,
                     double* __restrict__ g_save, double* __restrict__ l_save)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * d) return;
    const int64_t k = e / d;
    const int c = (int)(e - k * d);
    const uint64_t it = *iteration;
    p[k * ldp + c] = momentum_draw((uint64_t)e, it, seed, inv_mass ? inv_mass[e] : 1.0);
    if (x_save) {
        x_save[e] = x[k * ldx + c];
        g_save[e] = grad[e];
        if (e == 0) *l_save = *loglik;
    }
}

// the Metropolis test of transition *iteration; advances the counter
__global__ void hmc_decide_kernel(uint64_t seed, uint64_t* __restrict__ iteration,
                                  const double* __restrict__ energies, double* __restrict__ flag,
                                  double* __restrict__ stats, int64_t* __restrict__ accepted_total)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint64_t it = *iteration;
    const double h0 = energies[0], h1 = energies[1];
    const double lu = log(accept_draw(it, seed));
    const bool acc = lu < h0 - h1;  // false when the difference is NaN
    *flag = acc ? 1.0 : 0.0;
    if (stats) {
        stats[0] = h0;
        stats[1] = h1;
        stats[2] = lu;
        stats[3] = acc ? 1.0 : 0.0;
    }
    if (accepted_total && acc) *accepted_total += 1;
    *iteration = it + 1;
}

// a rejected proposal gives back the saved state
__global__ void __launch_bounds__(256)
    hmc_finish_kernel(int64_t n, int d, const double* __restrict__ flag, double* __restrict__ x,
                      int64_t ldx, double* __restrict__ grad, double* __restrict__ loglik,
                      const double* __restrict__ x_save, const double* __restrict__ g_save,
                      const double* __restrict__ l_save)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * d || *flag != 0.0) return;
    const int64_t k = e / d;
    const int c = (int)(e - k * d);
    x[k * ldx + c] = x_save[e];
    grad[e] = g_save[e];
    if (e == 0) *loglik = *l_save;
}

unsigned grid_of(int64_t count) { return (unsigned)((count + 255) / 256); }

}  // namespace

hipError_t launch_hmc_begin(int64_t n, int d, const double* inv_mass, uint64_t seed,
                            const uint64_t* iteration, double* p, int64_t ldp, const double* x,
                            int64_t ldx, const double* grad, const double* loglik, double* x_save,
                            double* g_save, double* l_save, hipStream_t s)
{
    if (n * d == 0) return hipSuccess;
    hipLaunchKernelGGL(hmc_begin_kernel, dim3(grid_of(n * d)), dim3(256), 0, s, n, d, inv_mass,
                       seed, iteration, p, ldp, x, ldx, grad, loglik, x_save, g_save, l_save);
    return hipGetLastError();
}

hipError_t launch_hmc_decide(uint64_t seed, uint64_t* iteration, const double* energies,
                             double* flag, double* stats, int64_t* accepted_total, hipStream_t s)
{
    hipLaunchKernelGGL(hmc_decide_kernel, dim3(1), dim3(64), 0, s, seed, iteration, energies, flag,
                       stats, accepted_total);
    return hipGetLastError();
}

hipError_t launch_hmc_finish(int64_t n, int d, const double* flag, double* x, int64_t ldx,
                             double* grad, double* loglik, const double* x_save,
                             const double* g_save, const double* l_save, hipStream_t s)
{
    if (n * d == 0) return hipSuccess;
    hipLaunchKernelGGL(hmc_finish_kernel, dim3(grid_of(n * d)), dim3(256), 0, s, n, d, flag, x,
                       ldx, grad, loglik, x_save, g_save, l_save);
    return hipGetLastError();
}

}  // namespace mds
