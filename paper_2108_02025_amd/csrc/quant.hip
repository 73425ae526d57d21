// Precision form: per-row scaled bfloat16 / OCP E4M3FN storage of A and the
// GEMV that streams it.
//
// The paper leaves the element width generic (section 2, S_data) and its
// GEMV is bound by the bytes of A (section 4.1 notes that bandwidth takes
// over at large sizes).  Storing A in 2 or 1 bytes per element cuts those
// bytes by 4x or 8x against binary64; x, c and the arithmetic stay binary32.
//
//   quantise: s_i from the row's largest magnitude, q_ij = RNE(fl32(a_ij/s_i))
//   gemv_q:   c_i += s_i * sum_j q_ij x_j, products and sums in binary32
//
// gemv_q has the row-dot shape of the binary64 GEMV: a group of G lanes owns
// a row, each lane loads 16 bytes of codes at a time (8 bfloat16 or 16 E4M3
// values) with non-temporal loads, decodes them in registers, and multiplies
// against x staged in LDS.  The scale is applied once per row, after the
// reduction.
#include <algorithm>

#include "sb_device.hpp"
#include "sb_internal.hpp"
#include "sb_quant.hpp"
#include "sb_rowdot.hpp"

// Build-time launch constants (overridable with -D for tuning sweeps).
#ifndef SB_GEMVQ_UNROLL_BF16
#define SB_GEMVQ_UNROLL_BF16 4
#endif
#ifndef SB_GEMVQ_UNROLL_E4M3
#define SB_GEMVQ_UNROLL_E4M3 8
#endif
#ifndef SB_GEMVQ_UNROLL_E4M3_XT
#define SB_GEMVQ_UNROLL_E4M3_XT 4
#endif
#ifndef SB_GEMVQ_MIN_WAVES
#define SB_GEMVQ_MIN_WAVES 4
#endif
#ifndef SB_GEMVQ_ROWS_BF16
#define SB_GEMVQ_ROWS_BF16 1
#endif
#ifndef SB_GEMVQ_ROWS_E4M3
#define SB_GEMVQ_ROWS_E4M3 1
#endif
#ifndef SB_GEMVQ_LOAD_NT
#define SB_GEMVQ_LOAD_NT 1
#endif
// Stage binary32 x with 16-byte loads where its chunk allows it (E4M3
// 47.6 -> 46.8 us, bfloat16 82.5 -> 81.3 us at 16384^2; the MX GEMVs'
// chunk-major layout gained nothing from it and stays per element).
#ifndef SB_STAGE_VEC
#define SB_STAGE_VEC 1
#endif
#ifndef SB_GEMVQ_WAVES_PER_CU
#define SB_GEMVQ_WAVES_PER_CU 32
#endif
// x above 40 KiB: threads per workgroup, and workgroups per compute unit.
// One workgroup per unit (x staged once per unit, half as many rows
// streaming at once) measured faster than two.
#ifndef SB_GEMVQ_NT_BIG_BF16
#define SB_GEMVQ_NT_BIG_BF16 512
#endif
#ifndef SB_GEMVQ_NT_BIG_E4M3
#define SB_GEMVQ_NT_BIG_E4M3 512
#endif
#ifndef SB_GEMVQ_BIG_WGS_PER_CU
#define SB_GEMVQ_BIG_WGS_PER_CU 1
#endif

namespace sb {

constexpr bool kGemvQNT = SB_GEMVQ_LOAD_NT;

template <bool BF16>
__global__ __launch_bounds__(256) void quantize_rows_kernel(int64_t m, int64_t n, const float* A,
                                                            int64_t lda, void* Aq, int64_t ldq,
                                                            float* scales)
{
    __shared__ float red[4];
    __shared__ float s_sh;
    const int64_t i = blockIdx.x;
    const float* Ar = A + i * lda;
    float amax = 0.0f;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const float v = fabsf(Ar[j]);
        if (v == v && v > amax) amax = v;
    }
    // max over the workgroup (order-independent)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        s_sh = row_scale(BF16, mx);
        scales[i] = s_sh;
    }
    __syncthreads();
    const float s = s_sh;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const float v = Ar[j] / s;
        if (BF16) static_cast<uint16_t*>(Aq)[i * ldq + j] = bf16_encode(v);
        else static_cast<uint8_t*>(Aq)[i * ldq + j] = e4m3_encode(v);
    }
}

// ------------------------------------------------------------- decoding ---

struct GemvQArgs {
    int64_t m, n, ldq;
    const void* Aq;
    const float* scales;
    const float* x;
    float* c;
    float* partial;  // nsplit x m, or nullptr
    int64_t KC, RB;
    int64_t NP;  // rows not 16-byte aligned: slots per residue of the transposed x
};

// A lower bound on waves per SIMD caps the registers the compiler may use
// for the loads in flight and their decodes.  XT (rows not 16-byte aligned,
// R = 1): x staged transposed by residue, read by tile_dot_xt.
template <bool BF16, int G, int NT, int R, bool XT = false>
__global__ __launch_bounds__(NT, XT && !BF16 && G < 64 ? 3 : SB_GEMVQ_MIN_WAVES) void gemv_q_kernel(GemvQArgs a)
{
    static_assert(!XT || R == 1, "transposed x is read one row at a time");
    typedef Codes<BF16> C;
    typedef typename C::code_t code_t;
    // E4M3 rows against the transposed x with several rows per wave: 4 loads
    // in flight (their 16 slot offsets per lane leave no registers for 8);
    // one row per wave keeps the offsets in scalar registers and 8 loads
    constexpr int U = BF16 ? SB_GEMVQ_UNROLL_BF16
                           : (XT && G < 64 ? SB_GEMVQ_UNROLL_E4M3_XT : SB_GEMVQ_UNROLL_E4M3);
    constexpr int NW = NT / kWave, GW = kWave / G;
    extern __shared__ __align__(16) unsigned char smem[];
    float* xs = reinterpret_cast<float*>(smem);

    const int64_t s = blockIdx.y;
    const int64_t k0 = s * a.KC;
    const int64_t klen = min(a.n, k0 + a.KC) - k0;
    const float* xg = a.x + k0;
    if constexpr (XT)
        stage_to_lds<NT>(xg, klen, [&](int64_t t, float v) { xs[xt_slot<C::PER16>(t, a.NP)] = v; });
    else if (SB_STAGE_VEC && ((reinterpret_cast<uintptr_t>(xg) | (uintptr_t)(klen * 4)) & 15) == 0)
        stage_to_lds<NT>(reinterpret_cast<const v4f*>(xg), klen / 4,
                         [&](int64_t t, v4f v) { reinterpret_cast<v4f*>(xs)[t] = v; });
    else
        stage_to_lds<NT>(xg, klen, [&](int64_t t, float v) { xs[t] = v; });
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int g = lane / G, l = lane % G;
    const int64_t r0 = (int64_t)blockIdx.x * a.RB;
    const int64_t r1 = min(a.m, r0 + a.RB);
    const code_t* Q = static_cast<const code_t*>(a.Aq);

    auto finish = [&](int64_t row, float t) {
        t = group_sum<G>(t);
        if (l == 0) {
            if (a.partial) a.partial[s * a.m + row] = t;
            else a.c[row] = a.c[row] + a.scales[row] * t;
        }
    };
    int64_t row = r0 + (int64_t)(w * GW + g) * R;
    if constexpr (XT) {
        for (; row < r1; row += (int64_t)NW * GW)
            finish(row, tile_dot_xt<C, G, U, kGemvQNT, true, true>(Q + row * a.ldq + k0, klen, xs, a.NP, l));
        return;
    }
    for (; row + R <= r1; row += (int64_t)NW * GW * R) {
        float t[R];
        tile_dot<C, G, U, R, kGemvQNT, true, true>(Q + row * a.ldq + k0, a.ldq, klen, xs, l, t);
#pragma unroll
        for (int r = 0; r < R; ++r) finish(row + r, t[r]);
    }
    // rows of a last, partial tile
    for (; row < r1; ++row) {
        float t[1];
        tile_dot<C, G, U, 1, kGemvQNT, true, true>(Q + row * a.ldq + k0, a.ldq, klen, xs, l, t);
        finish(row, t[0]);
    }
}

__global__ __launch_bounds__(256) void gemv_q_finish_kernel(int64_t m, int64_t nsplit,
                                                            const float* partial,
                                                            const float* scales, float* c)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    c[i] = c[i] + scales[i] * ordered_split_sum(partial + i, nsplit, m);
}

// ---------------------------------------------------------------- plans ---

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

struct GemvQPlan {
    int G, NT;
    int64_t KC, nsplit, RB, NP;
    size_t lds, ws;
};

// xt: rows not 16-byte aligned, x transposed by residue (NP slots each)
static GemvQPlan plan_gemv_q(sb_dtype q, int64_t m, int64_t n, int R, bool xt = false)
{
    GemvQPlan p{};
    const int64_t P = q == SB_BF16 ? 8 : 16;
    if (n * 4 <= 128 * 1024) {
        p.nsplit = 1;
        p.KC = std::max<int64_t>(round_up(n, 4), 4);
    } else {
        p.KC = 8192;
        p.nsplit = ceil_div(n, p.KC);
    }
    p.NP = xt ? (ceil_div(p.KC, P) | 1) : 0;
    p.lds = xt ? (size_t)(P * p.NP * 4) : (size_t)round_up(p.KC * 4, 16);
    const bool big = p.lds > 40 * 1024;
    p.NT = p.lds > 80 * 1024 ? 1024 : (big ? (q == SB_BF16 ? SB_GEMVQ_NT_BIG_BF16 : SB_GEMVQ_NT_BIG_E4M3) : 256);
    const int64_t wpb = p.NT / 64;
    const int64_t bpc = std::max<int64_t>(
        1, std::min<int64_t>((160 * 1024) / (int64_t)p.lds,
                             big ? SB_GEMVQ_BIG_WGS_PER_CU : SB_GEMVQ_WAVES_PER_CU / wpb));
    const int64_t nvec = ceil_div(p.KC, P);
    int G = 64;
    // (the transposed E4M3 form takes fewer loads per lane below 64 lanes a row)
    const int64_t U = q == SB_BF16 ? SB_GEMVQ_UNROLL_BF16 : SB_GEMVQ_UNROLL_E4M3;
    const int64_t Usmall = q == SB_BF16 || !xt ? U : SB_GEMVQ_UNROLL_E4M3_XT;
    if (nvec < 64 * U)
        while (G > 4 && nvec < (int64_t)G * Usmall) G >>= 1;
    p.G = G;
    const int64_t pass = wpb * (64 / G) * R;
    const int64_t row_blocks = std::max<int64_t>(1, ceil_div(256 * bpc, p.nsplit));
    p.RB = round_up(std::max<int64_t>(1, ceil_div(m, row_blocks)), pass);
    p.ws = p.nsplit > 1 ? (size_t)(p.nsplit * m * 4) : 0;
    return p;
}

size_t gemv_q_ws_bytes(sb_dtype q, int64_t m, int64_t n) { return plan_gemv_q(q, m, n, 1).ws; }

template <bool BF16, int G, int NT, int R, bool XT>
static void launch_q(const GemvQArgs& a, dim3 grid, size_t lds, hipStream_t st)
{
    static const bool attr_set = [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gemv_q_kernel<BF16, G, NT, R, XT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        return true;
    }();
    (void)attr_set;
    hipLaunchKernelGGL((gemv_q_kernel<BF16, G, NT, R, XT>), grid, dim3(NT), lds, st, a);
}

template <bool BF16, int NT, int R, bool XT>
static bool dispatch_q_g(int G, const GemvQArgs& a, dim3 grid, size_t lds, hipStream_t st)
{
    switch (G) {
    case 4: launch_q<BF16, 4, NT, R, XT>(a, grid, lds, st); return true;
    case 8: launch_q<BF16, 8, NT, R, XT>(a, grid, lds, st); return true;
    case 16: launch_q<BF16, 16, NT, R, XT>(a, grid, lds, st); return true;
    case 32: launch_q<BF16, 32, NT, R, XT>(a, grid, lds, st); return true;
    case 64: launch_q<BF16, 64, NT, R, XT>(a, grid, lds, st); return true;
    }
    return false;
}

template <bool BF16, int R, bool XT = false>
static bool dispatch_q(int NT, int G, const GemvQArgs& a, dim3 grid, size_t lds, hipStream_t st)
{
    switch (NT) {
    case 256: return dispatch_q_g<BF16, 256, R, XT>(G, a, grid, lds, st);
    case 512: return dispatch_q_g<BF16, 512, R, XT>(G, a, grid, lds, st);
    case 1024: return dispatch_q_g<BF16, 1024, R, XT>(G, a, grid, lds, st);
    }
    return false;
}

sb_status run_gemv_q(sb_handle* h, sb_dtype q, int64_t m, int64_t n, const void* Aq, int64_t ldq,
                     const float* scales, const float* x, float* c)
{
    if (m == 0 || n == 0) return SB_OK;
    const int csize = q == SB_BF16 ? 2 : 1;
    // Row tiles need every row of a tile at the same 16-byte alignment.
    const bool rows_aligned = (ldq * csize) % 16 == 0;
    // Rows not all 16-byte aligned read x transposed (conflict-free LDS
    // reads at any row start).
    const bool xt = !rows_aligned || (reinterpret_cast<uintptr_t>(Aq) & 15) != 0;
    constexpr int RB16 = SB_GEMVQ_ROWS_BF16, RE4 = SB_GEMVQ_ROWS_E4M3;
    const int R = rows_aligned ? (q == SB_BF16 ? RB16 : RE4) : 1;
    const GemvQPlan p = plan_gemv_q(q, m, n, xt ? 1 : R, xt);
    if (p.ws > h->ws_bytes)
        return fail(h, SB_ENOMEM, "gemv_q needs %zu workspace bytes, handle has %zu", p.ws, h->ws_bytes);
    if (p.nsplit > 65535)
        return fail(h, SB_EUNSUPPORTED, "gemv_q: rows of %lld codes need %lld column splits (at most 65535)",
                    (long long)n, (long long)p.nsplit);
    GemvQArgs a{m, n, ldq, Aq, scales, x, c, p.nsplit > 1 ? static_cast<float*>(claim_ws(h)) : nullptr, p.KC, p.RB,
                p.NP};
    const dim3 grid((unsigned)ceil_div(m, p.RB), (unsigned)p.nsplit);
    bool ok;
    if (xt)
        ok = q == SB_BF16 ? dispatch_q<true, 1, true>(p.NT, p.G, a, grid, p.lds, h->stream)
                          : dispatch_q<false, 1, true>(p.NT, p.G, a, grid, p.lds, h->stream);
    else if (q == SB_BF16)
        ok = R == 1 ? dispatch_q<true, 1>(p.NT, p.G, a, grid, p.lds, h->stream)
                    : dispatch_q<true, RB16>(p.NT, p.G, a, grid, p.lds, h->stream);
    else
        ok = R == 1 ? dispatch_q<false, 1>(p.NT, p.G, a, grid, p.lds, h->stream)
                    : dispatch_q<false, RE4>(p.NT, p.G, a, grid, p.lds, h->stream);
    if (!ok) return fail(h, SB_EINTERNAL, "no gemv_q instance for NT=%d G=%d", p.NT, p.G);
    sb_status st = check_launch(h, "gemv_q_kernel");
    if (st != SB_OK || p.nsplit == 1) return st;
    hipLaunchKernelGGL(gemv_q_finish_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, h->stream,
                       m, p.nsplit, static_cast<const float*>(h->ws), scales, c);
    return check_launch(h, "gemv_q_finish_kernel");
}

sb_status run_quantize_rows(sb_handle* h, sb_dtype q, int64_t m, int64_t n, const float* A,
                            int64_t lda, void* Aq, int64_t ldq, float* scales)
{
    if (m == 0) return SB_OK;
    if (q == SB_BF16)
        hipLaunchKernelGGL(quantize_rows_kernel<true>, dim3((unsigned)m), dim3(256), 0, h->stream, m, n,
                           A, lda, Aq, ldq, scales);
    else
        hipLaunchKernelGGL(quantize_rows_kernel<false>, dim3((unsigned)m), dim3(256), 0, h->stream, m, n,
                           A, lda, Aq, ldq, scales);
    return check_launch(h, "quantize_rows_kernel");
}

}  // namespace sb
