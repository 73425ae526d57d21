// DOT kernels: alpha += x . y (plain, binary64 or binary32) and the
// compensated binary32 form.
//
// The paper's section 4.3 splits a large dot product into blocks of n_c
// elements (Algorithm 4), gives each block to a thread and combines the
// block results; the definition (section 3.1) adds the initial alpha last.
// Here the blocks are contiguous chunks of a fixed number of workgroups
// G = f(n): every workgroup streams its chunk with 16-byte non-temporal
// loads into per-lane accumulators, reduces them (wave butterfly, then the
// waves in order) and writes one partial sum; a second kernel with one
// workgroup adds the G partial sums in index order and finally adds the
// initial alpha.  The order depends only on n, so results are reproducible.
// Below a cutoff in operand bytes one workgroup does everything in a single
// launch (the small-problem form of section 4.3).
#include <algorithm>

#include "sb_device.hpp"
#include "sb_internal.hpp"

namespace sb {

// Build-time launch constants (overridable with -D for tuning sweeps).
#ifndef SB_DOT_UNROLL
#define SB_DOT_UNROLL 16
#endif
#ifndef SB_DOT_LOAD_NT
#define SB_DOT_LOAD_NT 1
#endif
#ifndef SB_DOT_BLOCKS
#define SB_DOT_BLOCKS 1024
#endif
#ifndef SB_DOT_SMALL_BYTES
#define SB_DOT_SMALL_BYTES (256 * 1024)
#endif
constexpr int kUnrollDot = SB_DOT_UNROLL;
constexpr bool kDotNT = SB_DOT_LOAD_NT;
constexpr int kSmallNT = 1024;   // threads of the single-workgroup path
constexpr int kUnrollSmall = 4;
// Default operand bytes (x and y together) at or below which the
// single-workgroup path runs.  Measured per call under graph replay on
// MI355X: one workgroup is faster up to 256 KiB (binary64 n = 16384: 3.6 us
// against 4.4 us for two launches) and slower from 512 KiB on.
const int64_t kDefaultDotSmallBytes = SB_DOT_SMALL_BYTES;

template <typename T>
struct DotArgs {
    int64_t n;
    const T* x;
    const T* y;
    T* partial;
    int64_t chunk;
};

// Sum of x[b0, b1) . y[b0, b1) over one workgroup: 16-byte loads, U in
// flight per lane and operand, per-lane accumulators, then the workgroup
// reduction.  The result is valid in thread 0.
template <typename T, int NT, int U, bool ALIGNED, bool NTL>
__device__ __forceinline__ T dot_range(const T* x, const T* y, int64_t b0, int64_t b1, T* red)
{
    constexpr int W = ALIGNED ? Vec<T>::W : 1;
    typedef typename std::conditional<ALIGNED, typename Vec<T>::type, T>::type V;

    const int64_t nv = (b1 - b0) / W;
    const V* xv = reinterpret_cast<const V*>(x + b0);
    const V* yv = reinterpret_cast<const V*>(y + b0);

    V acc = (V)0;
    int64_t v = threadIdx.x;
    for (; v + (U - 1) * NT < nv; v += U * NT) {
        V xa[U], ya[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xa[u] = ld_stream<NTL>(xv + v + u * NT);
            ya[u] = ld_stream<NTL>(yv + v + u * NT);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += xa[u] * ya[u];
    }
    for (; v < nv; v += NT) acc += ld_stream<NTL>(xv + v) * ld_stream<NTL>(yv + v);

    T t;
    if constexpr (W == 1) {
        t = acc;
    } else {
        t = acc[0];
#pragma unroll
        for (int q = 1; q < W; ++q) t += acc[q];
    }
    const int64_t t0 = b0 + nv * W;  // fewer than W elements remain
    if (threadIdx.x < b1 - t0) t += x[t0 + threadIdx.x] * y[t0 + threadIdx.x];
    return block_sum<NT>(t, red);
}

template <typename T, int NT, bool ALIGNED>
__global__ __launch_bounds__(NT) void dot_stage1_kernel(DotArgs<T> a)
{
    __shared__ T red[NT / kWave];
    const int64_t b0 = (int64_t)blockIdx.x * a.chunk;
    const int64_t b1 = min(a.n, b0 + a.chunk);
    const T t = dot_range<T, NT, kUnrollDot, ALIGNED, kDotNT>(a.x, a.y, b0, b1, red);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = t;
}

// Small problems (section 4.3's Algorithm 3: no parallel split below a
// cutoff): one workgroup reads both vectors and adds the initial alpha
// itself, so the whole operation is one launch with no workspace.  Plain
// loads: operands this small are often still in the caches.
template <typename T, bool ALIGNED>
__global__ __launch_bounds__(kSmallNT) void dot_small_kernel(int64_t n, const T* x, const T* y, T* alpha)
{
    __shared__ T red[kSmallNT / kWave];
    const T t = dot_range<T, kSmallNT, kUnrollSmall, ALIGNED, false>(x, y, 0, n, red);
    if (threadIdx.x == 0) alpha[0] = alpha[0] + t;
}

// alpha = alpha + (sum of partial[0..nparts) in a fixed order).
template <typename T>
__global__ __launch_bounds__(256) void dot_stage2_kernel(int64_t nparts, const T* partial, T* alpha)
{
    __shared__ T red[256 / kWave];
    T t = 0;
    for (int64_t i = threadIdx.x; i < nparts; i += 256) t += partial[i];
    t = block_sum<256>(t, red);
    if (threadIdx.x == 0) alpha[0] = alpha[0] + t;
}

// ------------------------------------------------------- compensated DOT ---
//
// Error-free transformations (Ogita, Rump and Oishi 2005):
//   TwoProduct(a, b): p = fl(a*b), e = fma(a, b, -p)        a*b = p + e exactly
//   TwoSum(a, b):     s = fl(a+b), z = s - a,
//                     e = (a - (s - z)) + (b - z)           a+b = s + e exactly
// Each lane carries a pair (s, c): the running sum and the running sum of
// the rounding errors.  Pairs merge as (s, t) = TwoSum(s1, s2), c = c1 + c2 + t
// at every level of the reduction, and the initial alpha joins last:
// (s', t) = TwoSum(alpha, s), alpha = s' + (c + t).

struct Pair {
    float s, c;
};

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e)
{
    s = add_rn(a, b);
    const float z = sub_rn(s, a);
    e = add_rn(sub_rn(a, sub_rn(s, z)), sub_rn(b, z));
}

__device__ __forceinline__ Pair pair_merge(Pair a, Pair b)
{
    Pair r;
    float t;
    two_sum(a.s, b.s, r.s, t);
    r.c = add_rn(add_rn(a.c, b.c), t);
    return r;
}

// One product folded into a pair.
__device__ __forceinline__ void pair_fma(Pair& p, float x, float y)
{
    const float h = mul_rn(x, y);
    const float r = __builtin_fmaf(x, y, -h);  // exact error of the product
    float s, q;
    two_sum(p.s, h, s, q);
    p.s = s;
    p.c = add_rn(p.c, add_rn(q, r));
}

__device__ __forceinline__ Pair pair_shfl_xor(Pair p, int off)
{
    Pair r;
    r.s = __shfl_xor(p.s, off, kWave);
    r.c = __shfl_xor(p.c, off, kWave);
    return r;
}

template <int NT>
__device__ __forceinline__ Pair pair_block_sum(Pair p, Pair* lds)
{
    constexpr int NW = NT / kWave;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) p = pair_merge(p, pair_shfl_xor(p, off));
    if (NW == 1) return p;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) lds[w] = p;
    __syncthreads();
    Pair t = p;
    if (threadIdx.x == 0) {
        t = lds[0];
#pragma unroll
        for (int k = 1; k < NW; ++k) t = pair_merge(t, lds[k]);
    }
    return t;
}

// Compensated sum of x[b0, b1) . y[b0, b1) over one workgroup (the pair is
// valid in thread 0).
template <int NT, int U, bool ALIGNED, bool NTL>
__device__ __forceinline__ Pair dot2_range(const float* x, const float* y, int64_t b0, int64_t b1,
                                           Pair* red)
{
    constexpr int W = ALIGNED ? 4 : 1;
    typedef typename std::conditional<ALIGNED, v4f, float>::type V;

    const int64_t nv = (b1 - b0) / W;
    const V* xv = reinterpret_cast<const V*>(x + b0);
    const V* yv = reinterpret_cast<const V*>(y + b0);

    Pair acc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = Pair{0.0f, 0.0f};
    int64_t v = threadIdx.x;
    for (; v + (U - 1) * NT < nv; v += U * NT) {
        V xa[U], ya[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xa[u] = ld_stream<NTL>(xv + v + u * NT);
            ya[u] = ld_stream<NTL>(yv + v + u * NT);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (W == 1) {
                pair_fma(acc[0], xa[u], ya[u]);
            } else {
#pragma unroll
                for (int q = 0; q < W; ++q) pair_fma(acc[q], xa[u][q], ya[u][q]);
            }
        }
    }
    for (; v < nv; v += NT) {
        const V xa = ld_stream<NTL>(xv + v), ya = ld_stream<NTL>(yv + v);
        if constexpr (W == 1) {
            pair_fma(acc[0], xa, ya);
        } else {
#pragma unroll
            for (int q = 0; q < W; ++q) pair_fma(acc[q], xa[q], ya[q]);
        }
    }
    const int64_t t0 = b0 + nv * W;
    if (threadIdx.x < b1 - t0) pair_fma(acc[0], x[t0 + threadIdx.x], y[t0 + threadIdx.x]);

    Pair p = acc[0];
#pragma unroll
    for (int q = 1; q < W; ++q) p = pair_merge(p, acc[q]);
    return pair_block_sum<NT>(p, red);
}

// alpha joins last: (s', t) = TwoSum(alpha, s), alpha = s' + (c + t).
__device__ __forceinline__ void pair_finish(float* alpha, Pair p)
{
    float s, t;
    two_sum(alpha[0], p.s, s, t);
    alpha[0] = add_rn(s, add_rn(p.c, t));
}

template <int NT, bool ALIGNED>
__global__ __launch_bounds__(NT) void dot2_stage1_kernel(int64_t n, const float* x, const float* y,
                                                         float* partial, int64_t chunk)
{
    __shared__ Pair red[NT / kWave];
    const int64_t b0 = (int64_t)blockIdx.x * chunk;
    const int64_t b1 = min(n, b0 + chunk);
    const Pair p = dot2_range<NT, kUnrollDot, ALIGNED, kDotNT>(x, y, b0, b1, red);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = p.s;
        partial[2 * blockIdx.x + 1] = p.c;
    }
}

// The single-workgroup form for small problems (see dot_small_kernel).
template <bool ALIGNED>
__global__ __launch_bounds__(kSmallNT) void dot2_small_kernel(int64_t n, const float* x, const float* y,
                                                             float* alpha)
{
    __shared__ Pair red[kSmallNT / kWave];
    const Pair p = dot2_range<kSmallNT, kUnrollSmall, ALIGNED, false>(x, y, 0, n, red);
    if (threadIdx.x == 0) pair_finish(alpha, p);
}

__global__ __launch_bounds__(256) void dot2_stage2_kernel(int64_t nparts, const float* partial,
                                                          float* alpha)
{
    __shared__ Pair red[256 / kWave];
    Pair p{0.0f, 0.0f};
    for (int64_t i = threadIdx.x; i < nparts; i += 256)
        p = pair_merge(p, Pair{partial[2 * i], partial[2 * i + 1]});
    p = pair_block_sum<256>(p, red);
    if (threadIdx.x == 0) pair_finish(alpha, p);
}

// ---------------------------------------------------------------- plans ---

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int64_t kMaxDotBlocks = SB_DOT_BLOCKS;  // default: 4 workgroups per compute unit

DotPlan plan_dot(int esize, int64_t n, int partial_values, int64_t small_bytes)
{
    DotPlan p{};
    if (n * esize * 2 <= small_bytes) {
        p.small = true;
        p.NT = kSmallNT;
        p.nblocks = 1;
        p.chunk = n;
        p.ws = 0;
        return p;
    }
    p.NT = 256;
    const int64_t step = (int64_t)p.NT * (16 / esize);  // elements per workgroup pass
    const int64_t want = ceil_div(n, step * kUnrollDot);
    p.nblocks = std::max<int64_t>(1, std::min<int64_t>(want, kMaxDotBlocks));
    p.chunk = ceil_div(ceil_div(n, p.nblocks), step) * step;
    p.nblocks = std::max<int64_t>(1, ceil_div(n, p.chunk));
    p.ws = (size_t)(p.nblocks * partial_values * esize);
    return p;
}

template <typename T>
static sb_status dot_typed(sb_handle* h, int64_t n, const T* x, const T* y, T* alpha)
{
    const DotPlan p = plan_dot(sizeof(T), n, 1, h->dot_small_bytes);
    if (p.ws > h->ws_bytes)
        return fail(h, SB_ENOMEM, "dot needs %zu workspace bytes, handle has %zu", p.ws, h->ws_bytes);
    const bool al = aligned16(x) && aligned16(y);
    if (p.small) {
        if (al) hipLaunchKernelGGL((dot_small_kernel<T, true>), dim3(1), dim3(kSmallNT), 0, h->stream, n, x, y, alpha);
        else hipLaunchKernelGGL((dot_small_kernel<T, false>), dim3(1), dim3(kSmallNT), 0, h->stream, n, x, y, alpha);
        return check_launch(h, "dot_small_kernel");
    }
    T* part = static_cast<T*>(claim_ws(h));
    DotArgs<T> a{n, x, y, part, p.chunk};
    if (al) hipLaunchKernelGGL((dot_stage1_kernel<T, 256, true>), dim3((unsigned)p.nblocks), dim3(256), 0, h->stream, a);
    else hipLaunchKernelGGL((dot_stage1_kernel<T, 256, false>), dim3((unsigned)p.nblocks), dim3(256), 0, h->stream, a);
    sb_status st = check_launch(h, "dot_stage1_kernel");
    if (st != SB_OK) return st;
    hipLaunchKernelGGL(dot_stage2_kernel<T>, dim3(1), dim3(256), 0, h->stream, p.nblocks,
                       static_cast<const T*>(part), alpha);
    return check_launch(h, "dot_stage2_kernel");
}

sb_status run_dot(sb_handle* h, sb_dtype dt, int64_t n, const void* x, const void* y, void* alpha)
{
    if (n == 0) return SB_OK;
    if (dt == SB_F64)
        return dot_typed<double>(h, n, static_cast<const double*>(x), static_cast<const double*>(y),
                                 static_cast<double*>(alpha));
    return dot_typed<float>(h, n, static_cast<const float*>(x), static_cast<const float*>(y),
                            static_cast<float*>(alpha));
}

sb_status run_dot2(sb_handle* h, int64_t n, const float* x, const float* y, float* alpha)
{
    if (n == 0) return SB_OK;
    const DotPlan p = plan_dot(sizeof(float), n, 2, h->dot_small_bytes);
    if (p.ws > h->ws_bytes)
        return fail(h, SB_ENOMEM, "dot2 needs %zu workspace bytes, handle has %zu", p.ws, h->ws_bytes);
    if (p.small) {
        if (aligned16(x) && aligned16(y))
            hipLaunchKernelGGL((dot2_small_kernel<true>), dim3(1), dim3(kSmallNT), 0, h->stream, n, x, y, alpha);
        else
            hipLaunchKernelGGL((dot2_small_kernel<false>), dim3(1), dim3(kSmallNT), 0, h->stream, n, x, y, alpha);
        return check_launch(h, "dot2_small_kernel");
    }
    float* part = static_cast<float*>(claim_ws(h));
    if (aligned16(x) && aligned16(y))
        hipLaunchKernelGGL((dot2_stage1_kernel<256, true>), dim3((unsigned)p.nblocks), dim3(256), 0,
                           h->stream, n, x, y, part, p.chunk);
    else
        hipLaunchKernelGGL((dot2_stage1_kernel<256, false>), dim3((unsigned)p.nblocks), dim3(256), 0,
                           h->stream, n, x, y, part, p.chunk);
    sb_status st = check_launch(h, "dot2_stage1_kernel");
    if (st != SB_OK) return st;
    hipLaunchKernelGGL(dot2_stage2_kernel, dim3(1), dim3(256), 0, h->stream, p.nblocks,
                       static_cast<const float*>(part), alpha);
    return check_launch(h, "dot2_stage2_kernel");
}

}  // namespace sb
