// mds_rng.h -- device random draws of the HMC transition.
//
// Counter-based generator Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011): each of ten
// rounds multiplies counter words 0 and 2 by two 32-bit constants, keeps the
// high and low halves of the 64-bit products and mixes them with the other
// two words and the key; the key advances by two Weyl increments between
// rounds.  Draw k of transition `it` under `seed` is the block with counter
// (k_lo, k_hi, it_lo, it_hi) and key (seed_lo, seed_hi); a uniform in the open
// interval (0, 1) takes 26 bits from each of two output words (52 bits, exact
// in FP64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mds {

struct Philox4 {
    uint32_t r[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
    constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += kWeyl0;
            k1 += kWeyl1;
        }
        const uint32_t lo0 = kMul0 * c0, hi0 = __umulhi(kMul0, c0);
        const uint32_t lo1 = kMul1 * c2, hi1 = __umulhi(kMul1, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return Philox4{{c0, c1, c2, c3}};
}

__device__ __forceinline__ Philox4 draw_block(uint64_t k, uint64_t it, uint64_t seed)
{
    return philox4x32_10((uint32_t)k, (uint32_t)(k >> 32), (uint32_t)it, (uint32_t)(it >> 32),
                         (uint32_t)seed, (uint32_t)(seed >> 32));
}

// ((a >> 6) 2^26 + (b >> 6) + 1/2) 2^-52, in (0, 1)
__device__ __forceinline__ double uniform_open(uint32_t a, uint32_t b)
{
    return ((double)(a >> 6) * 67108864.0 + (double)(b >> 6) + 0.5) * 0x1p-52;
}

// momentum element e: Box-Muller on block e / 2, cosine branch for even e
__device__ __forceinline__ double momentum_draw(uint64_t e, uint64_t it, uint64_t seed,
                                                double inv_mass)
{
    const Philox4 b = draw_block(e >> 1, it, seed);
    const double u1 = uniform_open(b.r[0], b.r[1]);
    const double u2 = uniform_open(b.r[2], b.r[3]);
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 6.28318530717958647692 * u2;
    const double z = (e & 1) ? rad * sin(ang) : rad * cos(ang);
    return z / sqrt(inv_mass);
}

// the acceptance uniform of transition `it`: block k = 2^63
__device__ __forceinline__ double accept_draw(uint64_t it, uint64_t seed)
{
    const Philox4 b = draw_block((uint64_t)1 << 63, it, seed);
    return uniform_open(b.r[0], b.r[1]);
}

}  // namespace mds
