// Wave-level lane exchanges of gfx950 and the transposing butterfly built
// from them: the sum over a wave's 64 lanes of eight values per lane, for
// eight rows at once, without an LDS round trip.  Shared by the kernels whose
// lanes own fixed columns of a row (x held in registers) and so must reduce
// every row across the wave.
#pragma once

#include <stdint.h>

#include "sb_device.hpp"

namespace sb {

// Lane exchanges in the vector ALU (no LDS round trip):
//  swap32(a, b): the upper 32 lanes of a trade places with the lower 32
//                lanes of b (gfx950 v_permlane32_swap);
//  swap16(a, b): in each half wave, lanes 16..31 of a trade places with
//                lanes 0..15 of b (gfx950 v_permlane16_swap);
//  dpp<CTRL>(v): v as seen through a DPP lane pattern (row_ror, half
//                mirror, quad permutations; rows of 16 lanes).
__device__ __forceinline__ void swap32(uint32_t& a, uint32_t& b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}
__device__ __forceinline__ void swap16(uint32_t& a, uint32_t& b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}
template <bool S32>
__device__ __forceinline__ void swap_halves(float& a, float& b)
{
    uint32_t x = __float_as_uint(a), y = __float_as_uint(b);
    if constexpr (S32) swap32(x, y);
    else swap16(x, y);
    a = __uint_as_float(x);
    b = __uint_as_float(y);
}
template <bool S32>
__device__ __forceinline__ void swap_halves(double& a, double& b)
{
    const uint64_t x = (uint64_t)__double_as_longlong(a), y = (uint64_t)__double_as_longlong(b);
    uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32), yl = (uint32_t)y, yh = (uint32_t)(y >> 32);
    if constexpr (S32) {
        swap32(xl, yl);
        swap32(xh, yh);
    } else {
        swap16(xl, yl);
        swap16(xh, yh);
    }
    a = __longlong_as_double((long long)(((uint64_t)xh << 32) | xl));
    b = __longlong_as_double((long long)(((uint64_t)yh << 32) | yl));
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const uint64_t x = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
constexpr int kDppRowRor8 = 0x128, kDppHalfMirror = 0x141, kDppQuadXor1 = 0xB1, kDppQuadXor2 = 0x4E;

// Wave sum of p[0..8) for eight rows: returns, in lanes 8k .. 8k+7, the
// sum over all 64 lanes of p[k].  Exchanges at lane distance 32 and 16
// keep half of the rows each (the lanes of one half take rows 4..7, then
// 2..3 of what is left), distance 8 keeps one row, and three DPP steps sum
// the eight lanes that hold it.
template <typename T>
__device__ __forceinline__ T wave_sum8(const T (&p)[8], int lane)
{
    T q4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        T lo = p[k], hi = p[4 + k];
        swap_halves<true>(lo, hi);   // lanes 0..31: p[k] of lane + 32; 32..63: p[4 + k] of lane - 32
        q4[k] = lo + hi;             // row k (lanes 0..31) or 4 + k (lanes 32..63)
    }
    T q2[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        T lo = q4[k], hi = q4[2 + k];
        swap_halves<false>(lo, hi);
        q2[k] = lo + hi;             // row 4*b5 + 2*b4 + k
    }
    const bool b3 = lane & 8;
    const T mine = b3 ? q2[1] : q2[0];
    T q = mine + dpp<kDppRowRor8>(b3 ? q2[0] : q2[1]);  // row 4*b5 + 2*b4 + b3 = lane / 8
    q += dpp<kDppHalfMirror>(q);     // lane i of 8: i + (7 - i)
    q += dpp<kDppQuadXor1>(q);
    q += dpp<kDppQuadXor2>(q);
    return q;
}

}  // namespace sb
