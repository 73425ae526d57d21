// Two-sided GEMV: c += A x and d += A^T y in one pass over A.
//
// The paper (sections 4.1, 4.2 and the analysis of section 4.3) finds GEMV
// and its relatives bound by memory operations, not by arithmetic.  A
// caller that needs both products of one matrix (bidiagonalisation, the
// BLAS Technical Forum's fused GEMVT) pays for reading A twice with two
// calls; here every element of A is loaded once and feeds both sums, so the
// pair moves half the bytes.
//
// On a row-major view M (rows x cols, leading dimension ld) the kernel
// computes
//     out_r[i] += sum_j M_ij vc[j]      (row-dot, vc has cols entries)
//     out_c[j] += sum_i M_ij vr[i]      (col-axpy, vr has rows entries)
// A workgroup owns a band of NW*64*W columns (each wave 64*W of them, each
// lane W consecutive columns held with their vc values in registers) and a
// band of RS rows.  Per row a lane forms the W products with vc (its share
// of that row's dot) and adds M_ij vr[i] into its W column accumulators.
// The row shares are reduced eight rows at a time across the wave by a
// transposing butterfly (after the exchanges at lane distances 32, 16 and
// 8, lane 8k holds the partial of row k from all 64 lanes: 10 exchanges
// instead of 48, all of them gfx950 lane swaps or DPP moves in the vector
// ALU, so a wave returns to loading A without an LDS round trip), then
// across the waves in LDS in wave order.  Column bands
// and row bands beyond the first write partial sums that a second kernel
// adds in band order before adding the initial outputs.  Every output has
// one owner and the order depends only on the shape: results are
// reproducible bit for bit.
#include <stdint.h>

#include <algorithm>

#include "sb_device.hpp"
#include "sb_internal.hpp"
#include "sb_wave.hpp"

namespace sb {

#ifndef SB_GEMV2_LOAD_NT
#define SB_GEMV2_LOAD_NT 1
#endif
// Workgroups are sized so that one round fills the chip: measured faster
// than two rounds, whose extra workgroup starts and row-band partials cost
// more than the load balance they buy.  Eight waves per compute unit (one
// workgroup of at most eight waves) beat sixteen: fewer rows stream at once.
#ifndef SB_GEMV2_WAVES_PER_CU
#define SB_GEMV2_WAVES_PER_CU 8
#endif
#ifndef SB_GEMV2_MAX_WAVES
#define SB_GEMV2_MAX_WAVES 8
#endif
constexpr bool kGemv2NT = SB_GEMV2_LOAD_NT;
#ifndef SB_GEMV2_ROWS
#define SB_GEMV2_ROWS 8
#endif
constexpr int kRows2 = SB_GEMV2_ROWS;  // rows in flight per wave: 8 or 16, reduced in groups of 8
static_assert(kRows2 % 8 == 0, "rows are reduced in groups of eight");

template <typename T>
struct Gemv2Args {
    int64_t rows, cols, ld;
    const T* M;
    const T* vc;    // cols entries, multiplies along a row
    const T* vr;    // rows entries, multiplies down a column
    T* out_r;       // rows entries
    T* out_c;       // cols entries
    T* part_r;      // ncb x rows partial row sums, or nullptr when ncb == 1
    T* part_c;      // nsplit x cols partial column sums, or nullptr when nsplit == 1
    int64_t RS;     // rows per row band (multiple of kRows2)
    int64_t nsplit; // row bands
};

// W consecutive elements from p: one 16-byte load when aligned, else W
// element loads (the column coverage of a lane is the same either way).
template <typename T, bool ALIGNED>
__device__ __forceinline__ void load_w(const T* p, T (&v)[Vec<T>::W])
{
    constexpr int W = Vec<T>::W;
    if constexpr (ALIGNED) {
        const typename Vec<T>::type t = ld_stream<kGemv2NT>(reinterpret_cast<const typename Vec<T>::type*>(p));
#pragma unroll
        for (int q = 0; q < W; ++q) v[q] = t[q];
    } else {
#pragma unroll
        for (int q = 0; q < W; ++q) v[q] = ld_stream<kGemv2NT>(p + q);
    }
}

template <typename T, int NW, bool ALIGNED>
__global__ __launch_bounds__(NW * kWave) void gemv2_kernel(Gemv2Args<T> a)
{
    constexpr int W = Vec<T>::W;
    constexpr int U = kRows2;
    constexpr int CW = kWave * W;
    extern __shared__ __align__(16) unsigned char smem[];
    T* red = reinterpret_cast<T*>(smem);  // [NW][RS] per-wave row partials

    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t wcol = ((int64_t)blockIdx.x * NW + w) * CW;  // first column of this wave
    const int64_t j0 = wcol + lane * W;
    const int nvalid = j0 >= a.cols ? 0 : (int)min<int64_t>(W, a.cols - j0);
    const bool wave_full = wcol + CW <= a.cols;

    T xv[W];
#pragma unroll
    for (int q = 0; q < W; ++q) xv[q] = q < nvalid ? a.vc[j0 + q] : T(0);

    // Row bands blockIdx.y, blockIdx.y + gridDim.y, ...
    for (int64_t s = blockIdx.y; s < a.nsplit; s += gridDim.y) {
        const int64_t i0 = s * a.RS, i1 = min(a.rows, i0 + a.RS);
        T acc[W];
#pragma unroll
        for (int q = 0; q < W; ++q) acc[q] = 0;

        // `full`: every lane of the wave has W columns and the batch has U
        // rows (wave-uniform, so the exchanges always see all 64 lanes).
        auto batch = [&](int64_t i, auto full) {
            T p[U];
            if constexpr (decltype(full)::value) {
                T av[U][W];
                T yv[U];
                // wave-uniform row base (scalar registers) plus a small
                // per-lane offset
                const T* wbase = a.M + i * a.ld + wcol;
                const int loff = lane * W;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    load_w<T, ALIGNED>(wbase + u * a.ld + loff, av[u]);
                    yv[u] = a.vr[i + u];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    T t = av[u][0] * xv[0];
#pragma unroll
                    for (int q = 1; q < W; ++q) t += av[u][q] * xv[q];
                    p[u] = t;
#pragma unroll
                    for (int q = 0; q < W; ++q) acc[q] += av[u][q] * yv[u];
                }
            } else {
                // ragged edge: element loads of the valid columns and rows
                const int nr = (int)min<int64_t>(U, i1 - i);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    p[u] = 0;
                    if (u < nr) {
                        const T yu = a.vr[i + u];
                        const T* row = a.M + (i + u) * a.ld + j0;
                        T t = 0;
#pragma unroll
                        for (int q = 0; q < W; ++q) {
                            if (q < nvalid) {
                                const T av = row[q];
                                t += av * xv[q];
                                acc[q] += av * yu;
                            }
                        }
                        p[u] = t;
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < U; g += 8) {
                const T(&pg)[8] = *reinterpret_cast<const T(*)[8]>(p + g);
                const T r = wave_sum8(pg, lane);
                const int k = g + (lane >> 3);
                if ((lane & 7) == 0 && i + k < i1) red[w * a.RS + (i - i0) + k] = r;
            }
        };

        int64_t i = i0;
        if (wave_full) {
            for (; i + U <= i1; i += U) batch(i, std::true_type{});
        } else {
            for (; i + U <= i1; i += U) batch(i, std::false_type{});
        }
        if (i < i1) batch(i, std::false_type{});

        // column sums of this row band
#pragma unroll
        for (int q = 0; q < W; ++q) {
            if (q < nvalid) {
                if (a.part_c) a.part_c[s * a.cols + j0 + q] = acc[q];
                else a.out_c[j0 + q] = a.out_c[j0 + q] + acc[q];
            }
        }
        __syncthreads();
        // row sums of this column band: waves in order
        for (int64_t t = threadIdx.x; t < i1 - i0; t += NW * kWave) {
            T v = red[t];
#pragma unroll
            for (int k = 1; k < NW; ++k) v += red[k * a.RS + t];
            if (a.part_r) a.part_r[(int64_t)blockIdx.x * a.rows + i0 + t] = v;
            else a.out_r[i0 + t] = a.out_r[i0 + t] + v;
        }
        __syncthreads();  // red is rewritten by the next band
    }
}

// Adds the band partial sums in band order, then the initial outputs.
template <typename T>
__global__ __launch_bounds__(256) void gemv2_finish_kernel(int64_t rows, int64_t cols, int64_t ncb,
                                                           int64_t nsplit, const T* part_r,
                                                           const T* part_c, T* out_r, T* out_c)
{
    // the first ceil(rows/256) workgroups finish out_r, the rest out_c
    const int64_t rb = (rows + 255) / 256;
    if ((int64_t)blockIdx.x < rb) {
        const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
        if (part_r && i < rows) out_r[i] = out_r[i] + ordered_split_sum<16>(part_r + i, ncb, rows);
    } else {
        const int64_t j = ((int64_t)blockIdx.x - rb) * 256 + threadIdx.x;
        if (part_c && j < cols) out_c[j] = out_c[j] + ordered_split_sum<16>(part_c + j, nsplit, cols);
    }
}

// ---------------------------------------------------------------- plans ---

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

constexpr int64_t kCUs2 = 256;                 // MI355X compute units
constexpr int64_t kMaxRedBytes = 64 * 1024;    // LDS for the per-wave row partials
constexpr int64_t kMaxGridY = 65535;           // row bands beyond it loop inside the kernel

Gemv2Plan plan_gemv2(int esize, int64_t rows, int64_t cols)
{
    Gemv2Plan p{};
    const int64_t CW = 64 * (16 / esize);
    p.NW = 1;  // waves per workgroup: enough for the columns, at most 16
    while (p.NW < SB_GEMV2_MAX_WAVES && p.NW * CW < cols) p.NW *= 2;
    p.ncb = ceil_div(cols, p.NW * CW);
    const int64_t target = kCUs2 * SB_GEMV2_WAVES_PER_CU / p.NW;  // workgroups filling the chip
    int64_t ns = ceil_div(target, p.ncb);
    ns = std::max<int64_t>(1, std::min<int64_t>(ns, rows / 64));
    p.RS = round_up(ceil_div(rows, ns), kRows2);
    p.RS = std::min<int64_t>(p.RS, kMaxRedBytes / (p.NW * esize));
    p.nsplit = ceil_div(rows, p.RS);
    p.lds = (size_t)(p.NW * p.RS * esize);
    const size_t wr = p.ncb > 1 ? (size_t)(p.ncb * rows * esize) : 0;
    p.ws_c_offset = (wr + 255) / 256 * 256;
    p.ws = p.ws_c_offset + (p.nsplit > 1 ? (size_t)(p.nsplit * cols * esize) : 0);
    return p;
}

template <typename T, int NW, bool AL>
static void launch2(const Gemv2Args<T>& a, dim3 grid, size_t lds, hipStream_t st)
{
    static const bool attr_set = [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gemv2_kernel<T, NW, AL>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxRedBytes);
        return true;
    }();
    (void)attr_set;
    hipLaunchKernelGGL((gemv2_kernel<T, NW, AL>), grid, dim3(NW * kWave), lds, st, a);
}

template <typename T>
static sb_status gemv2_typed(sb_handle* h, int64_t rows, int64_t cols, const T* M, int64_t ld, const T* vc,
                             const T* vr, T* out_r, T* out_c)
{
    const Gemv2Plan p = plan_gemv2(sizeof(T), rows, cols);
    if (p.ws > h->ws_bytes)
        return fail(h, SB_ENOMEM, "gemv2 needs %zu workspace bytes, handle has %zu", p.ws, h->ws_bytes);
    if (p.ncb > 0x7FFFFFFF || ceil_div(rows, 256) + ceil_div(cols, 256) > ((int64_t)1 << 23))
        return fail(h, SB_EUNSUPPORTED, "gemv2: %lld x %lld exceeds the launch grid", (long long)rows, (long long)cols);
    unsigned char* ws = static_cast<unsigned char*>(p.ws ? claim_ws(h) : h->ws);
    Gemv2Args<T> a{rows, cols, ld, M, vc, vr, out_r, out_c,
                   p.ncb > 1 ? reinterpret_cast<T*>(ws) : nullptr,
                   p.nsplit > 1 ? reinterpret_cast<T*>(ws + p.ws_c_offset) : nullptr, p.RS, p.nsplit};
    const bool al = aligned16(M) && ((ld * (int64_t)sizeof(T)) % 16 == 0);
    const dim3 grid((unsigned)p.ncb, (unsigned)std::min<int64_t>(p.nsplit, kMaxGridY));
    switch (p.NW) {
    case 1: al ? launch2<T, 1, true>(a, grid, p.lds, h->stream) : launch2<T, 1, false>(a, grid, p.lds, h->stream); break;
    case 2: al ? launch2<T, 2, true>(a, grid, p.lds, h->stream) : launch2<T, 2, false>(a, grid, p.lds, h->stream); break;
    case 4: al ? launch2<T, 4, true>(a, grid, p.lds, h->stream) : launch2<T, 4, false>(a, grid, p.lds, h->stream); break;
    case 8: al ? launch2<T, 8, true>(a, grid, p.lds, h->stream) : launch2<T, 8, false>(a, grid, p.lds, h->stream); break;
    default: al ? launch2<T, 16, true>(a, grid, p.lds, h->stream) : launch2<T, 16, false>(a, grid, p.lds, h->stream); break;
    }
    sb_status st = check_launch(h, "gemv2_kernel");
    if (st != SB_OK || (p.ncb == 1 && p.nsplit == 1)) return st;
    hipLaunchKernelGGL(gemv2_finish_kernel<T>, dim3((unsigned)(ceil_div(rows, 256) + ceil_div(cols, 256))), dim3(256), 0,
                       h->stream, rows, cols, p.ncb, p.nsplit, static_cast<const T*>(a.part_r),
                       static_cast<const T*>(a.part_c), out_r, out_c);
    return check_launch(h, "gemv2_finish_kernel");
}

sb_status run_gemv2(sb_handle* h, sb_dtype dt, int64_t rows, int64_t cols, const void* M, int64_t ld,
                    const void* vc, const void* vr, void* out_r, void* out_c)
{
    if (rows == 0 || cols == 0) return SB_OK;
    if (dt == SB_F64)
        return gemv2_typed<double>(h, rows, cols, static_cast<const double*>(M), ld, static_cast<const double*>(vc),
                                   static_cast<const double*>(vr), static_cast<double*>(out_r),
                                   static_cast<double*>(out_c));
    return gemv2_typed<float>(h, rows, cols, static_cast<const float*>(M), ld, static_cast<const float*>(vc),
                              static_cast<const float*>(vr), static_cast<float*>(out_r), static_cast<float*>(out_c));
}

}  // namespace sb
