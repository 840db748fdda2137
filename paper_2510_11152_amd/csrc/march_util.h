// Lane-level helpers of the 2D march kernels (wave strips and block tiles): a lane holds
// a cell pair (2k, 2k + 1) of a 128-column window, and x-neighbours come from the
// adjacent lane by a DPP lane shift.
#pragma once
#include <hip/hip_runtime.h>

namespace fas {

// Lane i receives the value of lane i - 1 (wave_shr:1) or of lane i + 1 (wave_shl:1);
// the lane without a source receives 0.
constexpr int kShr1 = 0x138;  // wave_shr:1
constexpr int kShl1 = 0x130;  // wave_shl:1

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

template <typename T>
struct Pair;
template <>
struct Pair<double> {
    using V = double2;
};
template <>
struct Pair<float> {
    using V = float2;
};

// Index g of a periodic axis of n cells, wrapped into [0, n).
__device__ __forceinline__ int wrap(int g, int n)
{
    int w = g < 0 ? g + n : g - n;
    if (w < 0 || w >= n) w = ((g % n) + n) % n;
    return w;
}

// Value for a cell with xb / yb boundary faces across x / y: A (none), B (one), C (two).
template <typename T>
__device__ __forceinline__ T sel3(bool xb, bool yb, T A, T B, T C)
{
    return yb ? (xb ? C : B) : (xb ? B : A);
}

}  // namespace fas
