// Device-side building blocks shared by the streaming kernels (gfx950,
// wave64): 16-byte vector types, streaming loads/stores, and the
// deterministic wave / workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sb {

typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// 16-byte vector of T and its width.
template <typename T> struct Vec;
template <> struct Vec<double> { typedef v2d type; static constexpr int W = 2; };
template <> struct Vec<float> { typedef v4f type; static constexpr int W = 4; };

constexpr int kWave = 64;

// Loads of operands that are read exactly once (A, C, DOT's x and y) use the
// non-temporal hint so they stream past L2 and MALL instead of evicting the
// reused vector (x of GEMV).  NT selects the hint at compile time.
template <bool NT = true, typename V>
__device__ __forceinline__ V ld_stream(const V* p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT = true, typename V>
__device__ __forceinline__ void st_stream(V* p, V v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Copy n elements of a vector from global memory into LDS (put(t, v) stores
// element t), SU loads in flight per thread: a plain strided loop waits for
// each load before the next, which at 16 or 32 elements per thread made the
// staging of x a visible fixed cost of every GEMV call.  The caller
// synchronises the workgroup afterwards.
#ifndef SB_STAGE_UNROLL
#define SB_STAGE_UNROLL 16
#endif
template <int NT, int SU = SB_STAGE_UNROLL, typename T, typename F>
__device__ __forceinline__ void stage_to_lds(const T* __restrict__ src, int64_t n, F put)
{
    for (int64_t base = 0; base < n; base += (int64_t)SU * NT) {
        T v[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int64_t t = base + (int64_t)u * NT + threadIdx.x;
            v[u] = t < n ? src[t] : T(0);
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int64_t t = base + (int64_t)u * NT + threadIdx.x;
            if (t < n) put(t, v[u]);
        }
    }
}

// Separately rounded multiply / add / subtract.  Contraction into fused
// multiply-add is switched off inside each helper, so the operation keeps
// its own rounding even after inlining next to an addition (the default
// contraction mode would otherwise fuse x*y + c).  Used by GER, whose
// definition rounds the elementary product before the addition, and by the
// error-free transformations of the compensated DOT.
__device__ __forceinline__ double mul_rn(double a, double b)
{
#pragma clang fp contract(off)
    return a * b;
}
__device__ __forceinline__ float mul_rn(float a, float b)
{
#pragma clang fp contract(off)
    return a * b;
}
__device__ __forceinline__ double add_rn(double a, double b)
{
#pragma clang fp contract(off)
    return a + b;
}
__device__ __forceinline__ float add_rn(float a, float b)
{
#pragma clang fp contract(off)
    return a + b;
}
__device__ __forceinline__ float sub_rn(float a, float b)
{
#pragma clang fp contract(off)
    return a - b;
}

// Butterfly sum over groups of G consecutive lanes (G a power of two <= 64).
// Every lane of a group ends with the same value; the order of additions is
// fixed, so the result is deterministic.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum over a workgroup of NT threads, result valid in thread 0.  Waves
// reduce with the butterfly, then wave 0 adds the wave totals in wave order.
// `lds` must hold NT/64 values.  Contains __syncthreads().
template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T* lds)
{
    constexpr int NW = NT / kWave;
    v = group_sum<kWave>(v);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (NW == 1) return v;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    T t = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NW; ++k) t += lds[k];
    }
    return t;
}

// p[0] + p[stride] + ... + p[(ns - 1) * stride], added in order of the
// index (so the bits do not depend on how the loads are scheduled), with
// the loads issued AHEAD at a time before their additions, the last batch
// predicated: split partial sums were just written and sit in L2, where a
// chain of dependent loads would cost one L2 latency per split.
template <int AHEAD = 8, typename T>
__device__ __forceinline__ T ordered_split_sum(const T* p, int64_t ns, int64_t stride)
{
    T t = p[0];
    for (int64_t s = 1; s < ns; s += AHEAD) {
        T v[AHEAD];
#pragma unroll
        for (int u = 0; u < AHEAD; ++u) v[u] = s + u < ns ? p[(s + u) * stride] : T(0);
#pragma unroll
        for (int u = 0; u < AHEAD; ++u)
            if (s + u < ns) t += v[u];
    }
    return t;
}

}  // namespace sb
