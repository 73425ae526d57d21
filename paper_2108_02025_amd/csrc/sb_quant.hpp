// Row quantisation building blocks (bfloat16 and OCP E4M3FN encoders and
// the per-row scale), shared by the quantiser and the serving loop's
// operand generator so both produce identical codes.
#pragma once

#include "sb_device.hpp"

namespace sb {

// ------------------------------------------------------------- encoding ---

__device__ __forceinline__ uint32_t f32_bits(float f) { return __float_as_uint(f); }

// binary32 -> bfloat16, round to nearest even on the bit pattern; NaN
// becomes the canonical quiet NaN with the input's sign.
__device__ __forceinline__ uint16_t bf16_encode(float v)
{
    const uint32_t u = f32_bits(v);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)(((u >> 16) & 0x8000u) | 0x7FC0u);
    const uint32_t bias = 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)((u + bias) >> 16);
}

// Round-to-nearest-even right shift of a significand; carries propagate
// into the caller's exponent field naturally.
__device__ __forceinline__ uint32_t rne_shift(uint32_t v, int sh)
{
    const uint32_t q = v >> sh, rem = v & ((1u << sh) - 1u), half = 1u << (sh - 1);
    return q + ((rem > half || (rem == half && (q & 1u))) ? 1u : 0u);
}

// binary32 -> OCP E4M3FN (bias 7, 3 fraction bits, max 448, no infinity),
// round to nearest even, magnitudes >= 448 saturate to 448, NaN -> S.1111.111.
__device__ __forceinline__ uint8_t e4m3_encode(float v)
{
    const uint32_t u = f32_bits(v);
    const uint32_t sign = (u >> 24) & 0x80u;
    const uint32_t a = u & 0x7FFFFFFFu;
    if (a > 0x7F800000u) return (uint8_t)(sign | 0x7Fu);
    if (a >= 0x43E00000u) return (uint8_t)(sign | 0x7Eu);  // 448 = 1.75 * 2^8
    const int e = (int)(a >> 23) - 127;
    if (e < -6) {
        // E4M3 subnormals: value k * 2^-9 with k = RNE(v * 2^9).
        if (e < -10) return (uint8_t)sign;  // below 2^-10: rounds to zero
        const uint32_t mant = (a & 0x7FFFFFu) | 0x800000u;  // v = mant * 2^(e-23)
        return (uint8_t)(sign | rne_shift(mant, 14 - e));
    }
    // Normal: keep 3 of the 23 fraction bits; a carry bumps the exponent.
    const uint32_t base = ((uint32_t)(e + 7) << 3) | ((a & 0x7FFFFFu) >> 20);
    const uint32_t rem = a & 0xFFFFFu;
    uint32_t code = base + ((rem > 0x80000u || (rem == 0x80000u && (base & 1u))) ? 1u : 0u);
    if (code > 0x7Eu) code = 0x7Eu;
    return (uint8_t)(sign | code);
}

// Per-row scale: bfloat16 uses the power of two at or below amax; E4M3
// uses amax / 448.  Rows with amax 0 or infinite get 1.
__device__ __forceinline__ float row_scale(bool bf16, float amax)
{
    const uint32_t a = f32_bits(amax);
    if (a == 0u || a >= 0x7F800000u) return 1.0f;
    if (bf16) {
        if (a >= 0x00800000u) return __uint_as_float(a & 0x7F800000u);
        return __uint_as_float(1u << (31 - __clz((int)a)));  // subnormal: top set bit
    }
    const float s = amax / 448.0f;
    return s == 0.0f ? 1.0f : s;
}

// ------------------------------------------------------------ MX formats ---
// OCP Microscaling: blocks of 32 elements share an E8M0 scale 2^(code-127).

// binary32 -> OCP E2M1 (FP4; magnitudes 0, 0.5, 1, 1.5, 2, 3, 4, 6, no NaN
// or infinity): the code counts the rounding boundaries that |v| passes.  A
// value on a boundary is a tie and goes to the even code, so the test is
// ">=" where the code above is even and ">" where it is odd; past 5 the
// magnitude saturates to 6.  The sign bit is kept.
__device__ __forceinline__ uint8_t e2m1_encode(float v)
{
    const float a = fabsf(v);
    const uint32_t code = (uint32_t)(a > 0.25f) + (uint32_t)(a >= 0.75f) + (uint32_t)(a > 1.25f) +
                          (uint32_t)(a >= 1.75f) + (uint32_t)(a > 2.5f) + (uint32_t)(a >= 3.5f) +
                          (uint32_t)(a > 5.0f);
    return (uint8_t)(((f32_bits(v) >> 28) & 8u) | code);
}

// E8M0 code of a block whose largest magnitude is the finite amax:
// floor(log2 amax) - emax + 127, clamped to [0, 254]; 0 when amax is 0.
// emax is the exponent of the element format's largest value (8 for E4M3,
// 2 for E2M1), so amax / 2^(code-127) lands in [2^emax, 2^(emax+1)).
__device__ __forceinline__ int mx_scale_code(float amax, int emax)
{
    const uint32_t a = f32_bits(amax);
    if (a == 0u) return 0;
    // normal: the exponent field; subnormal (a * 2^-149): the top set bit
    const int e = a >= 0x00800000u ? (int)(a >> 23) - 127 : -118 - __clz((int)a);
    return min(max(e - emax + 127, 0), 254);
}

}  // namespace sb
