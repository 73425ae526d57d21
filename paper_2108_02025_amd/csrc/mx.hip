// Microscaled storage of A (OCP Microscaling Formats v1.0): MXFP8 (E4M3
// elements) and MXFP4 (E2M1 elements), blocks of 32 consecutive elements of
// a row sharing one E8M0 scale X = 2^(code - 127).
//
// The paper's GEMV is bound by the bytes of A (sections 4.1 and 4.3; the
// element width is its generic S_data).  Per-row scaled bfloat16 and E4M3
// cut those bytes by 4x and 8x against binary64; block-scaled E4M3 costs
// 1 + 1/32 bytes per element and E2M1 1/2 + 1/32, with a scale that follows
// the data every 32 elements instead of once per row.
//
//   quantise: per block, code = clamp(floor(log2 amax) - emax + 127, 0, 254)
//             (255 when the block holds a non-finite value), then
//             P_j = RNE_sat(a_j * 2^(127 - code))
//   gemv_mx:  c_i += sum over blocks of X_ib * sum_j P_ij x_j
//
// gemv_mx has the row-dot shape of the quantised GEMV: a group of G lanes
// owns a row, each lane loads 16 bytes of codes (16 E4M3 or 32 E2M1
// values, half a block or one block) with non-temporal loads, decodes them
// with gfx950's packed conversions, multiplies against x staged in LDS, and
// scales its partial sum of the block by X with one ldexp (exact for a
// power of two, so it equals scaling every element).  Rows of codes must
// start on 16-byte boundaries (Q 16-byte aligned, ldq a multiple of 16).
#include <algorithm>

#include "sb_device.hpp"
#include "sb_internal.hpp"
#include "sb_quant.hpp"

#ifndef SB_GEMVMX_TOUCH_SCALES
#define SB_GEMVMX_TOUCH_SCALES 1
#endif
#ifndef SB_GEMVMX_UNROLL_FP8
#define SB_GEMVMX_UNROLL_FP8 8
#endif
#ifndef SB_GEMVMX_UNROLL_FP4
#define SB_GEMVMX_UNROLL_FP4 8
#endif
#ifndef SB_GEMVMX_MIN_WAVES
#define SB_GEMVMX_MIN_WAVES 4
#endif
#ifndef SB_GEMVMX_LOAD_NT
#define SB_GEMVMX_LOAD_NT 1
#endif
#ifndef SB_GEMVMX_WAVES_PER_CU
#define SB_GEMVMX_WAVES_PER_CU 32
#endif
#ifndef SB_GEMVMX_NT_BIG
#define SB_GEMVMX_NT_BIG 1024
#endif
// x above 40 KiB: one workgroup of 1024 threads per compute unit.
#ifndef SB_GEMVMX_BIG_WGS_PER_CU
#define SB_GEMVMX_BIG_WGS_PER_CU 1
#endif
#ifndef SB_GEMVMX_UNROLL_BIG
#define SB_GEMVMX_UNROLL_BIG 4
#endif
#ifndef SB_GEMVMX_STAGE_MAX
#define SB_GEMVMX_STAGE_MAX (128 * 1024)
#endif

namespace sb {

// 16-byte loads in flight per lane: a 1024-thread workgroup (x above 40 KiB,
// one workgroup per compute unit) keeps fewer per lane than the 256-thread
// ones of shorter rows, several of which share a compute unit.
constexpr int mx_unroll(bool fp4, int nt)
{
    return nt >= 1024 ? SB_GEMVMX_UNROLL_BIG : (fp4 ? SB_GEMVMX_UNROLL_FP4 : SB_GEMVMX_UNROLL_FP8);
}

constexpr bool kGemvMxNT = SB_GEMVMX_LOAD_NT;

// ------------------------------------------------------------ quantiser ---

// One workgroup per row, 256 elements per pass: each half wave holds one
// block, reduces its largest magnitude and a non-finite flag with a
// butterfly, and encodes its 32 elements.
template <bool FP4>
__global__ __launch_bounds__(256) void quantize_mx_kernel(int64_t n, const float* A, int64_t lda, uint8_t* Q,
                                                          int64_t ldq, uint8_t* S, int64_t lds)
{
    constexpr int emax = FP4 ? 2 : 8;
    const int64_t i = blockIdx.x;
    for (int64_t base = 0; base < n; base += 256) {
        const int64_t e = base + threadIdx.x;
        const bool in = e < n;
        const float v = in ? A[i * lda + e] : 0.0f;
        int bad = (in && !isfinite(v)) ? 1 : 0;
        float amax = bad ? 0.0f : fabsf(v);
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) {
            amax = fmaxf(amax, __shfl_xor(amax, off, kWave));
            bad |= __shfl_xor(bad, off, kWave);
        }
        const int code = bad ? 255 : mx_scale_code(amax, emax);
        uint32_t cv = 0;
        if (code != 255) {
            const float sv = ldexpf(v, 127 - code);  // exact: a power-of-two scaling
            cv = FP4 ? e2m1_encode(sv) : e4m3_encode(sv);
        }
        if constexpr (FP4) {
            const uint32_t odd = __shfl_xor(cv, 1, kWave);
            if (in && (e & 1) == 0) Q[i * ldq + (e >> 1)] = (uint8_t)(cv | ((e + 1 < n ? odd : 0u) << 4));
        } else {
            if (in) Q[i * ldq + e] = (uint8_t)cv;
        }
        if (in && (e & 31) == 0) S[i * lds + (e >> 5)] = (uint8_t)code;
    }
}

// ------------------------------------------------------------- decoding ---

template <bool FP4> struct Mx;
template <> struct Mx<false> {  // E4M3 elements, one byte each
    static constexpr int P = 16;   // elements per 16-byte load (half a block)
    static constexpr int PD = 4;   // elements per dword
    __device__ static void dword(uint32_t d, float (&f)[4])
    {
        const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)d, false);
        const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)d, true);
        f[0] = lo[0];
        f[1] = lo[1];
        f[2] = hi[0];
        f[3] = hi[1];
    }
    __device__ static float one(const uint8_t* row, int64_t e) { return __builtin_amdgcn_cvt_f32_fp8((int)row[e], 0); }
};
template <> struct Mx<true> {  // E2M1 elements, element 2k in the low nibble of byte k
    static constexpr int P = 32;   // one block per 16-byte load
    static constexpr int PD = 8;
    __device__ static void dword(uint32_t d, float (&f)[8])
    {
        // gfx950 packed FP4 conversion (unit scale: the block scale is
        // applied to the block's partial sum)
        const auto b0 = __builtin_amdgcn_cvt_scalef32_pk_f32_fp4(d, 1.0f, 0);
        const auto b1 = __builtin_amdgcn_cvt_scalef32_pk_f32_fp4(d, 1.0f, 1);
        const auto b2 = __builtin_amdgcn_cvt_scalef32_pk_f32_fp4(d, 1.0f, 2);
        const auto b3 = __builtin_amdgcn_cvt_scalef32_pk_f32_fp4(d, 1.0f, 3);
        f[0] = b0[0];
        f[1] = b0[1];
        f[2] = b1[0];
        f[3] = b1[1];
        f[4] = b2[0];
        f[5] = b2[1];
        f[6] = b3[0];
        f[7] = b3[1];
    }
    __device__ static float one(const uint8_t* row, int64_t e)
    {
        const auto r = __builtin_amdgcn_cvt_scalef32_pk_f32_fp4((uint32_t)row[e >> 1], 1.0f, 0);
        return (e & 1) ? r[1] : r[0];
    }
};

// t * 2^(code - 127); the E8M0 code 255 is NaN.
__device__ __forceinline__ float mx_scaled(float t, uint32_t code)
{
    return code == 255u ? __builtin_nanf("") : ldexpf(t, (int)code - 127);
}

// x in LDS, chunk-major: the 16-byte chunk q (elements 4q .. 4q+3) of code
// vector v (elements v*P .. v*P+P-1) sits at float offset (q * NVC + v) * 4,
// NVC = vectors in the staged segment.  The lanes of a group read the same
// chunk of consecutive vectors, so one read instruction touches consecutive
// 16-byte slots (no bank conflicts); a plain layout would put the lanes P*4
// bytes apart.
template <int P>
__device__ __forceinline__ int64_t xs_slot(int64_t e, int64_t NVC)
{
    return (((e % P) >> 2) * NVC + e / P) * 4 + (e & 3);
}

// Partial dot product of one row segment of klen elements (codes from Qr,
// block scales from Sr, both at the segment start) with the staged x, for
// lane l of a group of G lanes.
template <bool FP4, int G, int U>
__device__ __forceinline__ float mx_row_dot(const uint8_t* Qr, const uint8_t* Sr, int64_t klen, const float* xs,
                                            int64_t NVC, int l)
{
    typedef Mx<FP4> C;
    constexpr int P = C::P, PD = C::PD;
    const int64_t nv = klen / P;
    const v4u* Qv = reinterpret_cast<const v4u*>(Qr);
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    // one 16-byte vector: four dwords of codes against four (E4M3) or eight
    // (E2M1) values of x each, then the block scale
    auto step = [&](const v4u& wv, uint32_t sc, int64_t v, int slot) {
        float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float f[PD];
            C::dword(wv[k], f);
#pragma unroll
            for (int q = 0; q < PD; q += 4) {
                const int chunk = (k * PD + q) >> 2;
                const v4f xv = *reinterpret_cast<const v4f*>(xs + (chunk * NVC + v) * 4);
                part[0] += f[q] * xv[0];
                part[1] += f[q + 1] * xv[1];
                part[2] += f[q + 2] * xv[2];
                part[3] += f[q + 3] * xv[3];
            }
        }
        acc[slot] += mx_scaled((part[0] + part[1]) + (part[2] + part[3]), sc);
    };
    int64_t v = l;
    // full batches (as many as every lane of the group has), then the rest
    // in one predicated batch
    const int64_t vfull = nv / (U * G) * (U * G);
    for (; v < vfull; v += U * G) {
        v4u wv[U];
        uint32_t sc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            wv[u] = ld_stream<kGemvMxNT>(Qv + v + u * G);
            sc[u] = Sr[((v + u * G) * P) >> 5];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            step(wv[u], sc[u], v + u * G, u & 3);
            // keep each vector's decodes and LDS reads inside its step (the
            // loads above are already in flight)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (v < nv) {
        // fewer than U vectors remain for this lane: one predicated batch
        v4u wv[U];
        uint32_t sc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = v + u * G < nv;
            wv[u] = in ? ld_stream<kGemvMxNT>(Qv + v + u * G) : v4u{0, 0, 0, 0};
            sc[u] = in ? Sr[((v + u * G) * P) >> 5] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (v + u * G < nv) step(wv[u], sc[u], v + u * G, u & 3);
    }
    for (int64_t e = nv * P + l; e < klen; e += G)
        acc[1] += mx_scaled(C::one(Qr, e) * xs[xs_slot<P>(e, NVC)], Sr[e >> 5]);
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

struct GemvMxArgs {
    int64_t m, n, ldq, lds;  // strides in bytes
    const uint8_t* Q;
    const uint8_t* S;
    const float* x;
    float* c;
    float* partial;  // nsplit x m, or nullptr
    int64_t KC, RB;  // KC: columns per split, a multiple of 32
};

template <bool FP4, int G, int NT>
__global__ __launch_bounds__(NT, SB_GEMVMX_MIN_WAVES) void gemv_mx_kernel(GemvMxArgs a)
{
    constexpr int U = mx_unroll(FP4, NT);
    constexpr int NW = NT / kWave, GW = kWave / G;
    extern __shared__ __align__(16) unsigned char smem[];
    float* xs = reinterpret_cast<float*>(smem);

    constexpr int P = Mx<FP4>::P;
    const int64_t s = blockIdx.y;
    const int64_t k0 = s * a.KC;
    const int64_t klen = min(a.n, k0 + a.KC) - k0;
    const int64_t NVC = (klen + P - 1) / P;
    const int64_t r0 = (int64_t)blockIdx.x * a.RB;
    const int64_t r1 = min(a.m, r0 + a.RB);

    // Read one byte of every 64 of this workgroup's block scales (one load
    // per thread at most) before staging x, so that the row loop finds
    // them in L2: after other kernels have filled the caches, their first
    // reads would otherwise wait on HBM inside the loop.
    uint32_t touch = 0;
    {
        const int64_t sbytes = (klen + 31) / 32, per_row = (sbytes + 63) / 64;
        const int64_t i = threadIdx.x, row = r0 + i / per_row;
        if (SB_GEMVMX_TOUCH_SCALES && i < (r1 - r0) * per_row) touch = a.S[row * a.lds + k0 / 32 + (i % per_row) * 64];
    }
    stage_to_lds<NT>(a.x + k0, klen, [&](int64_t t, float v) { xs[xs_slot<P>(t, NVC)] = v; });
    __syncthreads();
    if (a.m < 0) a.c[0] = (float)touch;  // never taken (m >= 0): keeps the loads

    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int g = lane / G, l = lane % G;
    const int64_t qoff = FP4 ? k0 / 2 : k0;  // k0 is a multiple of 32
    for (int64_t row = r0 + w * GW + g; row < r1; row += NW * GW) {
        float t = mx_row_dot<FP4, G, U>(a.Q + row * a.ldq + qoff, a.S + row * a.lds + k0 / 32, klen, xs, NVC, l);
        t = group_sum<G>(t);
        if (l == 0) {
            if (a.partial) a.partial[s * a.m + row] = t;
            else a.c[row] = a.c[row] + t;
        }
    }
}

__global__ __launch_bounds__(256) void gemv_mx_finish_kernel(int64_t m, int64_t nsplit, const float* partial,
                                                             float* c)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    c[i] = c[i] + ordered_split_sum<16>(partial + i, nsplit, m);
}

// ---------------------------------------------------------------- plans ---

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

struct GemvMxPlan {
    int G, NT;
    int64_t KC, nsplit, RB;
    size_t lds, ws;
};

static GemvMxPlan plan_gemv_mx(bool fp4, int64_t m, int64_t n)
{
    GemvMxPlan p{};
    const int64_t P = fp4 ? 32 : 16;
    if (n * 4 <= SB_GEMVMX_STAGE_MAX) {
        p.nsplit = 1;
        p.KC = std::max<int64_t>(round_up(n, 4), 4);
    } else {
        p.KC = 8192;  // 32 KiB of x, a whole number of blocks
        p.nsplit = ceil_div(n, p.KC);
    }
    p.lds = (size_t)(round_up(p.KC, P) * 4);  // chunk-major x: whole vectors
    const bool big = p.lds > 40 * 1024;
    p.NT = p.lds > 80 * 1024 ? 1024 : (big ? SB_GEMVMX_NT_BIG : 256);
    const int64_t wpb = p.NT / 64;
    const int64_t bpc = std::max<int64_t>(
        1, std::min<int64_t>((160 * 1024) / (int64_t)p.lds,
                             big ? SB_GEMVMX_BIG_WGS_PER_CU : SB_GEMVMX_WAVES_PER_CU / wpb));
    const int64_t nvec = ceil_div(p.KC, P);
    const int64_t U = mx_unroll(fp4, p.NT);
    int G = 64;
    while (G > 4 && nvec < (int64_t)G * U) G >>= 1;
    p.G = G;
    const int64_t pass = wpb * (64 / G);
    const int64_t row_blocks = std::max<int64_t>(1, ceil_div(256 * bpc, p.nsplit));
    p.RB = round_up(std::max<int64_t>(1, ceil_div(m, row_blocks)), pass);
    p.ws = p.nsplit > 1 ? (size_t)(p.nsplit * m * 4) : 0;
    return p;
}

size_t gemv_mx_ws_bytes(sb_dtype q, int64_t m, int64_t n)
{
    return plan_gemv_mx(q == SB_MXFP4_E2M1, m, n).ws;
}

template <bool FP4, int G, int NT>
static void launch_mx(const GemvMxArgs& a, dim3 grid, size_t lds, hipStream_t st)
{
    static const bool attr_set = [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gemv_mx_kernel<FP4, G, NT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        return true;
    }();
    (void)attr_set;
    hipLaunchKernelGGL((gemv_mx_kernel<FP4, G, NT>), grid, dim3(NT), lds, st, a);
}

template <bool FP4, int NT>
static bool dispatch_mx_g(int G, const GemvMxArgs& a, dim3 grid, size_t lds, hipStream_t st)
{
    switch (G) {
    case 4: launch_mx<FP4, 4, NT>(a, grid, lds, st); return true;
    case 8: launch_mx<FP4, 8, NT>(a, grid, lds, st); return true;
    case 16: launch_mx<FP4, 16, NT>(a, grid, lds, st); return true;
    case 32: launch_mx<FP4, 32, NT>(a, grid, lds, st); return true;
    case 64: launch_mx<FP4, 64, NT>(a, grid, lds, st); return true;
    }
    return false;
}

template <bool FP4>
static bool dispatch_mx(int NT, int G, const GemvMxArgs& a, dim3 grid, size_t lds, hipStream_t st)
{
    switch (NT) {
    case 256: return dispatch_mx_g<FP4, 256>(G, a, grid, lds, st);
    case 512: return dispatch_mx_g<FP4, 512>(G, a, grid, lds, st);
    case 1024: return dispatch_mx_g<FP4, 1024>(G, a, grid, lds, st);
    }
    return false;
}

sb_status run_quantize_mx(sb_handle* h, sb_dtype q, int64_t m, int64_t n, const float* A, int64_t lda, void* Q,
                          int64_t ldq, uint8_t* S, int64_t lds)
{
    if (m == 0 || n == 0) return SB_OK;
    if (m > 0x7FFFFFFF) return fail(h, SB_EUNSUPPORTED, "quantize_mx: more than 2^31-1 rows");
    uint8_t* Qb = static_cast<uint8_t*>(Q);
    if (q == SB_MXFP4_E2M1)
        hipLaunchKernelGGL(quantize_mx_kernel<true>, dim3((unsigned)m), dim3(256), 0, h->stream, n, A, lda, Qb, ldq, S, lds);
    else
        hipLaunchKernelGGL(quantize_mx_kernel<false>, dim3((unsigned)m), dim3(256), 0, h->stream, n, A, lda, Qb, ldq, S, lds);
    return check_launch(h, "quantize_mx_kernel");
}

sb_status run_gemv_mx(sb_handle* h, sb_dtype q, int64_t m, int64_t n, const void* Q, int64_t ldq, const uint8_t* S,
                      int64_t lds, const float* x, float* c)
{
    if (m == 0 || n == 0) return SB_OK;
    const bool fp4 = q == SB_MXFP4_E2M1;
    const GemvMxPlan p = plan_gemv_mx(fp4, m, n);
    if (p.ws > h->ws_bytes)
        return fail(h, SB_ENOMEM, "gemv_mx needs %zu workspace bytes, handle has %zu", p.ws, h->ws_bytes);
    if (p.nsplit > 65535)
        return fail(h, SB_EUNSUPPORTED, "gemv_mx: rows of %lld elements need %lld column splits (at most 65535)",
                    (long long)n, (long long)p.nsplit);
    GemvMxArgs a{m, n, ldq, lds, static_cast<const uint8_t*>(Q), S, x, c,
                 p.nsplit > 1 ? static_cast<float*>(claim_ws(h)) : nullptr, p.KC, p.RB};
    const dim3 grid((unsigned)ceil_div(m, p.RB), (unsigned)p.nsplit);
    const bool ok = fp4 ? dispatch_mx<true>(p.NT, p.G, a, grid, p.lds, h->stream)
                        : dispatch_mx<false>(p.NT, p.G, a, grid, p.lds, h->stream);
    if (!ok) return fail(h, SB_EINTERNAL, "no gemv_mx instance for NT=%d G=%d", p.NT, p.G);
    sb_status st = check_launch(h, "gemv_mx_kernel");
    if (st != SB_OK || p.nsplit == 1) return st;
    hipLaunchKernelGGL(gemv_mx_finish_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, h->stream, m, p.nsplit,
                       static_cast<const float*>(h->ws), c);
    return check_launch(h, "gemv_mx_finish_kernel");
}

}  // namespace sb
