// mds_wave.h -- in-wave sums by DPP lane exchanges, shared by the sweep and
// the finalize kernels (gfx950, 64-wide waves).
#pragma once

#include <hip/hip_runtime.h>

namespace mds {

// Cross-lane sums by DPP (the VALU's lane-routing operand modifier): no LDS
// traffic and no address arithmetic, unlike a shuffle.  dpp<CTRL, ROWS>(v) is
// the value CTRL routes to this lane; lanes of rows that the mask ROWS leaves
// out read 0.
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]: lane ^ 1
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]: lane ^ 2
constexpr int kDppRowMirror = 0x140;   // lane 15 - l within a row of 16
constexpr int kDppHalfMirror = 0x141;  // lane 7 - l within each half row
constexpr int kDppBcast15 = 0x142;     // lane 15 of the row before
constexpr int kDppBcast31 = 0x143;     // lane 31

// ROWS = 0xF routes a value to every lane (the patterns used here never
// leave a row), so the lane's old value is not needed (bound_ctrl).
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ int dpp(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, ROWS == 0xF);
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(dpp<CTRL, ROWS>(__float_as_int(v)));
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)dpp<CTRL, ROWS>((int)(unsigned)b);
    const unsigned hi = (unsigned)dpp<CTRL, ROWS>((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over each aligned group of G lanes (G = 4, 8 or 16); every lane of a
// group ends with the same value (each exchange adds two equal pairs of
// operands in either order).
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v)
{
    static_assert(G == 4 || G == 8 || G == 16, "group of 4, 8 or 16 lanes");
    v += dpp<kDppXor1>(v);
    v += dpp<kDppXor2>(v);
    if constexpr (G >= 8) v += dpp<kDppHalfMirror>(v);
    if constexpr (G >= 16) v += dpp<kDppRowMirror>(v);
    return v;
}

__device__ __forceinline__ int read_lane63(int v) { return __builtin_amdgcn_readlane(v, 63); }
__device__ __forceinline__ double read_lane63(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes in a fixed order, returned to every lane: row sums
// of 16, then row 1 += row 0 and row 3 += row 2, then row 3 += rows 0-1.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    v = group_sum<16>(v);
    v += dpp<kDppBcast15, 0xA>(v);
    v += dpp<kDppBcast31, 0xC>(v);
    return read_lane63(v);
}

}  // namespace mds
