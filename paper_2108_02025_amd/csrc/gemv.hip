// GEMV kernels: c += A x and c += A^T x on a row-major view of A.
//
// The paper's section 3.1 defines c_i as the sum of the products A_ij x_j
// with the initial c_i added last; section 4.2 (Algorithm 2) walks a
// row-major A row by row with stride one, and section 4.1 (Algorithm 1)
// walks a column-major A by blocks of columns, updating a short segment of
// c per block.  On the GPU the two access patterns become two kernels:
//
//  * row-dot (gemv_n_kernel): a group of G lanes owns one row and streams it
//    with 16-byte non-temporal loads; x for the current column split sits in
//    LDS; the group reduces with a butterfly and its first lane adds the
//    initial c_i (or writes a split partial).  Used for row-major N and
//    column-major T.
//  * col-axpy (gemv_t_kernel): each lane owns W consecutive outputs; the
//    waves of a workgroup take interleaved rows of one row split, x_i is
//    wave-uniform, partial column sums are combined across waves in LDS in
//    wave order.  This is Algorithm 1's micro-kernel shape (a contiguous
//    segment of the output updated over a block of the reduction index).
//    Used for row-major T and column-major N.  Rows that are not 16-byte
//    aligned: gemv_t_phase_kernel (binary32: the same 16-byte loads, one
//    accumulator set per row phase) or gemv_t_elem_kernel (binary64:
//    element loads).  Wide matrices with few rows: gemv_t_band_kernel (the
//    waves side by side, each walking every row).
//
// Splits (of columns for row-dot, of rows for col-axpy) write partial sums
// to the workspace and a second kernel adds them in split order (above 32
// splits: 64 in-order partial chains combined by a fixed butterfly), then
// adds the initial output.  No atomics anywhere: every output has one owner, and
// the summation order depends only on the shape, so results are
// reproducible bit for bit.
#include <algorithm>
#include <type_traits>

#include "sb_device.hpp"
#include "sb_internal.hpp"
#include "sb_rowdot.hpp"

namespace sb {

// Build-time launch constants (overridable with -D for tuning sweeps).
#ifndef SB_GEMV_N_UNROLL
#define SB_GEMV_N_UNROLL 16
#endif
#ifndef SB_GEMV_T_UNROLL
#define SB_GEMV_T_UNROLL 8
#endif
#ifndef SB_GEMV_LOAD_NT
#define SB_GEMV_LOAD_NT 1
#endif
#ifndef SB_GEMV_T_BLOCKS
#define SB_GEMV_T_BLOCKS 1024
#endif
#ifndef SB_GEMV_N_WAVES_PER_CU
#define SB_GEMV_N_WAVES_PER_CU 32
#endif
// x above 80 KiB (one workgroup per compute unit): 8 waves, each streaming
// one row with 16 loads in flight per lane, measured faster than 16 waves.
#ifndef SB_GEMV_N_NT_HUGE
#define SB_GEMV_N_NT_HUGE 512
#endif
#ifndef SB_GEMV_N_SPLIT_MIN_BYTES
#define SB_GEMV_N_SPLIT_MIN_BYTES (32ll << 20)
#endif
#ifndef SB_GEMV_T_SMALL_SPLITS
#define SB_GEMV_T_SMALL_SPLITS 2
#endif
constexpr int kUnrollN = SB_GEMV_N_UNROLL;  // 16-byte loads in flight per lane and row
// x above 80 KiB (8 waves per compute unit, whole rows of 10240+ binary64
// or 20480+ binary32 values): 32 loads in flight per lane
#ifndef SB_GEMV_N_UNROLL_HUGE
#define SB_GEMV_N_UNROLL_HUGE 32
#endif
constexpr int kUnrollNHuge = SB_GEMV_N_UNROLL_HUGE;
constexpr int kUnrollT = SB_GEMV_T_UNROLL;  // rows in flight per wave
// the phase kernel of unaligned binary32 rows: 4 rows in flight per wave
// (65537 x 4093: 193-195 -> 186 us against 8)
#ifndef SB_GEMV_T_PHASE_UNROLL
#define SB_GEMV_T_PHASE_UNROLL 4
#endif
constexpr bool kGemvNT = SB_GEMV_LOAD_NT;

template <typename T>
struct GemvNArgs {
    int64_t rows, cols, ld;
    const T* A;
    const T* x;
    T* c;
    T* partial;  // nsplit x rows, or nullptr when nsplit == 1
    int64_t KC;
    int64_t RB;
};

// SHIFT (rows not 16-byte aligned, x small enough): LDS holds W copies of
// the x chunk, copy h shifted left by h elements, KC elements apart, and a
// row whose first 16-byte boundary is h elements in reads copy h as
// aligned vectors (otherwise it reads x one element at a time: four LDS
// reads instead of one per binary32 vector).  PAIRS (binary32 rows not
// aligned, x too large for four copies but not for two): copies 0 and 1,
// and a row peeled by h reads copy h % 2 as 8-byte pairs.  Same arithmetic
// either way.
template <typename T, int G, int NT, bool ALIGNED, int U = kUnrollN, bool SHIFT = false, bool PAIRS = false>
__global__ __launch_bounds__(NT) void gemv_n_kernel(GemvNArgs<T> a)
{
    constexpr int NW = NT / kWave, GW = kWave / G;
    constexpr int W = Vec<T>::W;
    extern __shared__ __align__(16) unsigned char smem[];
    T* xs = reinterpret_cast<T*>(smem);

    const int64_t s = blockIdx.y;
    const int64_t k0 = s * a.KC;
    const int64_t klen = min(a.cols, k0 + a.KC) - k0;

    // Stage x[k0, k0 + klen) in LDS (read by every row of this workgroup).
    if constexpr (SHIFT) {
        stage_to_lds<NT>(a.x + k0, klen, [&](int64_t t, T v) {
#pragma unroll
            for (int h = 0; h < W; ++h)
                if (t >= h) xs[h * a.KC + t - h] = v;
        });
    } else if constexpr (PAIRS) {
        stage_to_lds<NT>(a.x + k0, klen, [&](int64_t t, T v) {
            xs[t] = v;
            if (t >= 1) xs[a.KC + t - 1] = v;
        });
    } else {
        stage_to_lds<NT>(a.x + k0, klen, [&](int64_t t, T v) { xs[t] = v; });
    }
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int g = lane / G, l = lane % G;
    const int64_t r0 = (int64_t)blockIdx.x * a.RB;
    const int64_t r1 = min(a.rows, r0 + a.RB);

    for (int64_t row = r0 + w * GW + g; row < r1; row += NW * GW) {
        T t = row_dot<T, G, U, ALIGNED, kGemvNT, true, SHIFT, true, PAIRS>(a.A + row * a.ld + k0, klen, xs, l, a.KC);
        t = group_sum<G>(t);
        if (l == 0) {
            if (a.partial) a.partial[s * a.rows + row] = t;
            else a.c[row] = a.c[row] + t;
        }
    }
}

// out[i] = out[i] + sum over splits of partial[s * len + i], splits in order.
// Deep splits (more than kWaveFinishSplits): one wave per output; lane l adds
// splits l, l + 64, ... in order (loads 8 ahead), then the lanes' sums are
// combined by a butterfly, a fixed order, so that no thread waits on a long
// chain of dependent loads (512 splits took 25-29 us one thread per output).
constexpr int64_t kWaveFinishSplits = 32;
template <typename T>
__global__ __launch_bounds__(256) void split_finish_wave_kernel(int64_t len, int64_t nsplit,
                                                                const T* partial, T* out)
{
    const int64_t i = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;  // wave-uniform
    const int lane = threadIdx.x & (kWave - 1);
    if (i >= len) return;
    T t = lane < nsplit ? ordered_split_sum<8>(partial + lane * len + i, (nsplit - lane + kWave - 1) / kWave,
                                               kWave * len)
                        : T(0);
    t = group_sum<kWave>(t);
    if (lane == 0) out[i] = out[i] + t;
}

template <typename T>
__global__ __launch_bounds__(256) void split_finish_kernel(int64_t len, int64_t nsplit,
                                                           const T* partial, T* out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    out[i] = out[i] + ordered_split_sum<16>(partial + i, nsplit, len);
}

template <typename T>
struct GemvTElemArgs {
    int64_t rows, cols, ld;
    const T* A;
    const T* x;
    T* c;
    T* partial;  // nsplit x cols, or nullptr when nsplit == 1
    int64_t RS;
};

template <typename T>
struct GemvTArgs {
    int64_t rows, cols, ld;
    const T* A;
    const T* x;
    T* c;
    T* partial;  // nsplit x cols, or nullptr when nsplit == 1
    int64_t RS;
};

template <typename T, int NT, bool ALIGNED>
__global__ __launch_bounds__(NT) void gemv_t_kernel(GemvTArgs<T> a)
{
    constexpr int W = ALIGNED ? Vec<T>::W : 1;
    typedef typename std::conditional<ALIGNED, typename Vec<T>::type, T>::type V;
    // rows in flight per wave: element loads (rows not 16-byte aligned) move
    // fewer bytes each, so keep more of them in flight
    constexpr int U = ALIGNED ? kUnrollT : 16 / sizeof(T) * kUnrollT;
    constexpr int NW = NT / kWave;
    constexpr int CW = kWave * W;
    __shared__ T red[NW][CW];

    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t j0 = (int64_t)blockIdx.x * CW + lane * W;
    const int64_t s = blockIdx.y;
    const int64_t i0 = s * a.RS, i1 = min(a.rows, i0 + a.RS);

    T acc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = 0;

    if (j0 + W <= a.cols) {
        int64_t i = i0 + w;
        for (; i + (U - 1) * NW < i1; i += U * NW) {
            V av[U];
            T xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                av[u] = ld_stream<kGemvNT>(reinterpret_cast<const V*>(a.A + (i + u * NW) * a.ld + j0));
                xv[u] = a.x[i + u * NW];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if constexpr (W == 1) {
                    acc[0] += av[u] * xv[u];
                } else {
#pragma unroll
                    for (int q = 0; q < W; ++q) acc[q] += av[u][q] * xv[u];
                }
            }
        }
        for (; i < i1; i += NW) {
            const V av = ld_stream<kGemvNT>(reinterpret_cast<const V*>(a.A + i * a.ld + j0));
            const T xv = a.x[i];
            if constexpr (W == 1) {
                acc[0] += av * xv;
            } else {
#pragma unroll
                for (int q = 0; q < W; ++q) acc[q] += av[q] * xv;
            }
        }
    } else if (j0 < a.cols) {
        const int rem = (int)(a.cols - j0);
        for (int64_t i = i0 + w; i < i1; i += NW) {
            const T xv = a.x[i];
            for (int q = 0; q < rem; ++q) acc[q] += a.A[i * a.ld + j0 + q] * xv;
        }
    }

#pragma unroll
    for (int q = 0; q < W; ++q) red[w][lane * W + q] = acc[q];
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int q = 0; q < W; ++q) {
            T t = red[0][lane * W + q];
#pragma unroll
            for (int k = 1; k < NW; ++k) t += red[k][lane * W + q];
            const int64_t j = j0 + q;
            if (j < a.cols) {
                if (a.partial) a.partial[s * a.cols + j] = t;
                else a.c[j] = a.c[j] + t;
            }
        }
    }
}

// Column-axpy for binary32 rows that are not 16-byte aligned, with the
// aligned kernel's 16-byte loads, column blocks and row splits.  Row i
// starts r_i elements past a 16-byte boundary (r_i < W, the same for the
// whole row), so the vector at index v of the row's aligned grid holds
// columns W*v - r_i + q (q < W): lane l's vector (v = 64*b + l in column
// block b) holds W - r_i of the lane's own columns and r_i of lane l - 1's.
// Each lane adds its vector's products into one of W accumulator sets,
// chosen by the row's phase r_i, and the columns are put together once,
// after the rows: lane l's column W*v + t takes, phase by phase, set r's
// position t + r if that is below W, else position t + r - W of lane
// l + 1's set r.  The last lane also loads the vector after its own (rows
// with r_i > 0) into a set of its own, whose first r_i positions close the
// block.  A column's sum is the sum over phases, in phase order, of its
// rows' products in row order per wave; then the waves in order, as in the
// aligned kernel.  Every loaded vector holds at least one column of its row
// (so it lies in a page of the matrix); elements outside the block's
// columns fall into positions that are dropped.  (Binary64 rows, two
// phases, run faster with element loads.)
#ifndef SB_GEMV_T_PHASE
#define SB_GEMV_T_PHASE 1
#endif
template <typename T>
__global__ __launch_bounds__(256) void gemv_t_phase_kernel(GemvTArgs<T> a)
{
    constexpr int W = Vec<T>::W;
    typedef typename Vec<T>::type V;
    constexpr int U = SB_GEMV_T_PHASE_UNROLL;
    constexpr int NW = 256 / kWave;
    constexpr int CW = kWave * W;
    __shared__ T red[NW][CW];

    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const bool last = lane == kWave - 1;
    const int64_t v = (int64_t)blockIdx.x * kWave + lane;  // this lane's vector of each row
    const int64_t s = blockIdx.y;
    const int64_t i0 = s * a.RS, i1 = min(a.rows, i0 + a.RS);

    T acc[W][W], ext[W][W];
#pragma unroll
    for (int r = 0; r < W; ++r) {
#pragma unroll
        for (int q = 0; q < W; ++q) acc[r][q] = ext[r][q] = 0;
    }
    // Loads of row i: the lane's vector (if it holds a column of the row)
    // and, for the last lane, the next one.
    auto load_row = [&](int64_t i, V& av, V& ev) -> int {
        const T* p = a.A + i * a.ld;
        const int r = __builtin_amdgcn_readfirstlane((int)((reinterpret_cast<uintptr_t>(p) & 15) / sizeof(T)));
        const V* b = reinterpret_cast<const V*>(p - r);
        av = v * W - r < a.cols ? ld_stream<kGemvNT>(b + v) : (V)0;
        ev = (last && r > 0 && (v + 1) * W - r < a.cols) ? ld_stream<kGemvNT>(b + v + 1) : (V)0;
        return r;
    };
    auto add_row = [&](int r, const V& av, const V& ev, T xv) {
#pragma unroll
        for (int ph = 0; ph < W; ++ph) {
            if (r == ph) {
#pragma unroll
                for (int q = 0; q < W; ++q) acc[ph][q] += av[q] * xv;
#pragma unroll
                for (int q = 0; q < ph; ++q) ext[ph][q] += ev[q] * xv;
            }
        }
    };

    int64_t i = i0 + w;
    for (; i + (U - 1) * NW < i1; i += U * NW) {
        V av[U], ev[U];
        T xv[U];
        int rr[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            rr[u] = load_row(i + u * NW, av[u], ev[u]);
            xv[u] = a.x[i + u * NW];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) add_row(rr[u], av[u], ev[u], xv[u]);
    }
    for (; i < i1; i += NW) {
        V av, ev;
        const int r = load_row(i, av, ev);
        add_row(r, av, ev, a.x[i]);
    }

    // Put the columns together: phase by phase, in phase order.
    T tot[W];
#pragma unroll
    for (int ph = 0; ph < W; ++ph) {
#pragma unroll
        for (int t = 0; t < W; ++t) {
            T part;
            if (t + ph < W) {
                part = acc[ph][t + ph];
            } else {
                const T nb = __shfl_down(acc[ph][t + ph - W], 1);
                part = last ? ext[ph][t + ph - W] : nb;
            }
            tot[t] = ph == 0 ? part : tot[t] + part;
        }
    }
#pragma unroll
    for (int t = 0; t < W; ++t) red[w][lane * W + t] = tot[t];
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int t = 0; t < W; ++t) {
            T sum = red[0][lane * W + t];
#pragma unroll
            for (int k = 1; k < NW; ++k) sum += red[k][lane * W + t];
            const int64_t j = v * W + t;
            if (j < a.cols) {
                if (a.partial) a.partial[s * a.cols + j] = sum;
                else a.c[j] = a.c[j] + sum;
            }
        }
    }
}

// Column-axpy for rows that are not 16-byte aligned (element loads): each
// wave owns 64 consecutive columns and walks every row of its split, the
// four waves of a workgroup side by side, so that the cache lines a row's
// 256-column stretch shares with its neighbours at the edges are fetched by
// one workgroup (row starts then fall anywhere in a line).  A lane adds its
// column's products in row order.
template <typename T>
__global__ __launch_bounds__(256) void gemv_t_elem_kernel(GemvTElemArgs<T> a)
{
    constexpr int U = 32;  // rows in flight per wave
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t j = (int64_t)blockIdx.x * 256 + w * kWave + lane;
    const int64_t s = blockIdx.y;
    const int64_t i0 = s * a.RS, i1 = min(a.rows, i0 + a.RS);
    if (j >= a.cols) return;  // no barriers below
    const T* Aj = a.A + j;
    T acc = 0;
    int64_t i = i0;
    for (; i + U - 1 < i1; i += U) {
        T av[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            av[u] = ld_stream<kGemvNT>(Aj + (i + u) * a.ld);
            xv[u] = a.x[i + u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += av[u] * xv[u];
    }
    if (i < i1) {
        T av[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = i + u < i1;
            av[u] = in ? ld_stream<kGemvNT>(Aj + (i + u) * a.ld) : T(0);
            xv[u] = in ? a.x[i + u] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u < i1) acc += av[u] * xv[u];
    }
    if (a.partial) a.partial[s * a.cols + j] = acc;
    else a.c[j] = a.c[j] + acc;
}

// Column-axpy for wide matrices with few rows (one row split): the four
// waves of a workgroup side by side, each owning 64 x W consecutive columns
// (one 16-byte vector per lane) and walking every row, 8 rows in flight; no
// cross-wave sum.  A workgroup then reads 4 KiB of each row at once, where
// the row-interleaved kernel reads 1 KiB of four rows, a whole row apart
// (2 MiB for 256 x 262144 binary64: 99 -> 88 us; binary32 50 -> 43 us).  A
// lane adds its columns' products in row order.
template <typename T>
__global__ __launch_bounds__(256) void gemv_t_band_kernel(GemvTArgs<T> a)
{
    constexpr int W = Vec<T>::W;
    typedef typename Vec<T>::type V;
    constexpr int U = kUnrollT;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t j0 = ((int64_t)blockIdx.x * (256 / kWave) + w) * kWave * W + lane * W;
    const int64_t i1 = a.rows;
    if (j0 >= a.cols) return;  // no barriers below
    T acc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = 0;
    if (j0 + W <= a.cols) {
        int64_t i = 0;
        for (; i + U - 1 < i1; i += U) {
            V av[U];
            T xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                av[u] = ld_stream<kGemvNT>(reinterpret_cast<const V*>(a.A + (i + u) * a.ld + j0));
                xv[u] = a.x[i + u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int q = 0; q < W; ++q) acc[q] += av[u][q] * xv[u];
            }
        }
        if (i < i1) {  // fewer than U rows left: one predicated batch
            V av[U];
            T xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in = i + u < i1;
                av[u] = in ? ld_stream<kGemvNT>(reinterpret_cast<const V*>(a.A + (i + u) * a.ld + j0)) : (V)0;
                xv[u] = in ? a.x[i + u] : T(0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (i + u < i1) {
#pragma unroll
                    for (int q = 0; q < W; ++q) acc[q] += av[u][q] * xv[u];
                }
            }
        }
    } else {
        // right edge: fewer than W columns left for this lane
        for (int64_t i = 0; i < i1; ++i) {
#pragma unroll
            for (int q = 0; q < W; ++q)
                if (j0 + q < a.cols) acc[q] += a.A[i * a.ld + j0 + q] * a.x[i];
        }
    }
#pragma unroll
    for (int q = 0; q < W; ++q)
        if (j0 + q < a.cols) a.c[j0 + q] = a.c[j0 + q] + acc[q];
}

// ---------------------------------------------------------------- plans ---

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

constexpr int64_t kCUs = 256;                  // MI355X compute units
constexpr int64_t kLdsPerCU = 160 * 1024;      // gfx950 LDS per compute unit
constexpr int64_t kMaxStagedX = 128 * 1024;    // x bytes staged whole before splitting
constexpr int64_t kSplitChunkBytes = 32 * 1024;
constexpr int64_t kSplitFloorBytes = 16 * 1024;  // smallest chunk the few-rows split goes down to
#ifndef SB_GEMV_N_SHIFTED_X_BYTES
#define SB_GEMV_N_SHIFTED_X_BYTES (80 * 1024)
#endif
constexpr int64_t kShiftedXBytes = SB_GEMV_N_SHIFTED_X_BYTES;  // LDS for shifted x copies (0: never)
// Side-by-side GEMV-T (gemv_t_band_kernel): aligned rows, no row split, at
// least 1024 column blocks of one wave (256 workgroups of four) and at most
// 1024 rows (measured: 256 and 512 rows gain 8-13%, more rows or fewer
// blocks leave too few waves walking too many rows).
constexpr int64_t kGemvTBandBlocks = 1024, kGemvTBandRows = 1024;

// Launch shape for a column chunk of KC elements (nsplit chunks per row).
static void shape_gemv_n(GemvNPlan& p, int esize, int64_t rows)
{
    const int W = 16 / esize;
    p.lds = (size_t)p.xcopies * (size_t)round_up(p.KC * esize, 16);
    p.NT = p.lds > 80 * 1024 ? SB_GEMV_N_NT_HUGE : (p.lds > 40 * 1024 ? 512 : 256);
    const int64_t waves_per_block = p.NT / 64;
    const int64_t bpc = std::max<int64_t>(1, std::min<int64_t>(kLdsPerCU / (int64_t)p.lds,
                                                              SB_GEMV_N_WAVES_PER_CU / waves_per_block));
    const int64_t nvec = ceil_div(p.KC, W);
    // Lanes per row: the fewest that leave kUnrollN vectors per lane, but
    // at least 8 (a 128-byte line per row and load instruction: with 4 lanes
    // a row, each instruction reads half of 16 lines; 262144 x 256 binary32
    // 51.1 -> 47.7 us, 524288 x 128 binary64 106 -> 94 us) unless a row has
    // fewer than 32 vectors (1048576 x 64 binary32: 4 lanes 64 us, 8 lanes 71).
    int G = 64;
    const int gmin = nvec >= 32 ? 8 : 4;
    while (G > gmin && nvec < (int64_t)G * kUnrollN) G >>= 1;
    p.G = G;
    const int64_t pass = waves_per_block * (64 / G);  // rows a workgroup covers at once
    const int64_t target = kCUs * bpc;
    const int64_t row_blocks = std::max<int64_t>(1, ceil_div(target, p.nsplit));
    p.RB = round_up(std::max<int64_t>(1, ceil_div(rows, row_blocks)), pass);
}

GemvNPlan plan_gemv_n(int esize, int64_t rows, int64_t cols, bool unaligned)
{
    GemvNPlan p{};
    p.xcopies = 1;
    const int W = 16 / esize;
    if (cols * esize <= kMaxStagedX) {
        p.nsplit = 1;
        p.KC = std::max<int64_t>(round_up(cols, W), W);
    } else {
        p.KC = kSplitChunkBytes / esize;
        p.nsplit = ceil_div(cols, p.KC);
    }
    shape_gemv_n(p, esize, rows);
    // Few long rows: with one group per row there are fewer waves than the
    // chip holds (16 per compute unit), so halve the column chunk until
    // there are enough; the partial sums then go through the second stage.
    // Only for operands large enough that the second launch pays off.
    if (rows * cols * esize >= SB_GEMV_N_SPLIT_MIN_BYTES) {
        while (ceil_div(rows * p.G, 64) * p.nsplit < kCUs * 16 && p.KC * esize > kSplitFloorBytes) {
            p.KC = round_up(ceil_div(p.KC, 2), W);
            p.nsplit = ceil_div(cols, p.KC);
            shape_gemv_n(p, esize, rows);
        }
    }
    // Rows not 16-byte aligned: shifted copies of x when W of them fit
    // kShiftedXBytes of LDS (x read as vectors; at most about 20 KiB of x).
    if (unaligned && p.nsplit == 1 && W * round_up(p.KC * esize, 16) <= kShiftedXBytes) {
        p.xcopies = W;
        shape_gemv_n(p, esize, rows);
    } else if (unaligned && esize == 4 && p.nsplit == 1 && 2 * round_up(p.KC * esize, 16) <= kMaxStagedX) {
        // binary32: two copies read as 8-byte pairs where four do not fit
        p.xcopies = 2;
        p.pairs = true;
        shape_gemv_n(p, esize, rows);
    }
    p.ws = p.nsplit > 1 ? (size_t)(p.nsplit * rows * esize) : 0;
    return p;
}

// Default largest row split replaced by the unsplit single-launch form.
// Measured per call under graph replay on MI355X: a 2-way split (128..191
// rows) is slower than 16 waves per column block (binary64 128 x 1024:
// 4.9 us against 4.0 us), a 3-way split about as fast, 4 ways and more
// faster (one compute unit then streams too many bytes).
const int64_t kDefaultGemvTSmallSplits = SB_GEMV_T_SMALL_SPLITS;

GemvTPlan plan_gemv_t(int esize, int64_t rows, int64_t cols, int64_t small_splits)
{
    GemvTPlan p{};
    p.NT = 256;
    const int64_t CW = 64 * (16 / esize);
    const int64_t ncb = std::max<int64_t>(1, ceil_div(cols, CW));
    const int64_t target = SB_GEMV_T_BLOCKS;
    int64_t ns = ceil_div(target, ncb);
    ns = std::min<int64_t>(ns, 512);
    ns = std::min<int64_t>(ns, std::max<int64_t>(1, rows / 64));
    ns = std::max<int64_t>(ns, 1);
    if (ns >= 2 && ns <= small_splits) {
        // Few rows (section 4's advice for small problems: fewer parallel
        // parts): one workgroup of 16 waves per column block has at least
        // the waves of a split of up to four ways, and needs no second
        // kernel and no workspace, so the call is a single launch.
        p.NT = 1024;
        p.RS = rows;
        p.nsplit = 1;
        p.ws = 0;
        return p;
    }
    p.RS = ceil_div(rows, ns);
    p.nsplit = ceil_div(rows, p.RS);
    p.ws = p.nsplit > 1 ? (size_t)(p.nsplit * cols * esize) : 0;
    return p;
}

// ------------------------------------------------------------- launchers ---

template <typename T, int G, int NT, bool AL, int U = kUnrollN, bool SH = false, bool PR = false>
static void launch_n(const GemvNArgs<T>& a, dim3 grid, size_t lds, hipStream_t st)
{
    static const bool attr_set = [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gemv_n_kernel<T, G, NT, AL, U, SH, PR>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsPerCU);
        return true;
    }();
    (void)attr_set;
    hipLaunchKernelGGL((gemv_n_kernel<T, G, NT, AL, U, SH, PR>), grid, dim3(NT), lds, st, a);
}

template <typename T, int NT, bool AL, bool SH, bool PR>
static bool dispatch_n_g(int G, const GemvNArgs<T>& a, dim3 grid, size_t lds, hipStream_t st)
{
    switch (G) {
    case 4: launch_n<T, 4, NT, AL, kUnrollN, SH, PR>(a, grid, lds, st); return true;
    case 8: launch_n<T, 8, NT, AL, kUnrollN, SH, PR>(a, grid, lds, st); return true;
    case 16: launch_n<T, 16, NT, AL, kUnrollN, SH, PR>(a, grid, lds, st); return true;
    case 32: launch_n<T, 32, NT, AL, kUnrollN, SH, PR>(a, grid, lds, st); return true;
    case 64: launch_n<T, 64, NT, AL, kUnrollN, SH, PR>(a, grid, lds, st); return true;
    }
    return false;
}

template <typename T, bool AL, bool SH = false, bool PR = false>
static bool dispatch_n(int NT, int G, const GemvNArgs<T>& a, dim3 grid, size_t lds, hipStream_t st)
{
    switch (NT) {  // the shapes shape_gemv_n picks (SB_GEMV_N_NT_HUGE goes through launch_n)
    case 256: return dispatch_n_g<T, 256, AL, SH, PR>(G, a, grid, lds, st);
    case 512: return dispatch_n_g<T, 512, AL, SH, PR>(G, a, grid, lds, st);
    }
    return false;
}

// out[i] += the nsplit partial sums of output i (len outputs).
template <typename T>
static void launch_split_finish(hipStream_t st, int64_t len, int64_t nsplit, const T* partial, T* out)
{
    if (nsplit > kWaveFinishSplits)
        hipLaunchKernelGGL(split_finish_wave_kernel<T>, dim3((unsigned)ceil_div(len, 256 / kWave)), dim3(256), 0, st,
                           len, nsplit, partial, out);
    else
        hipLaunchKernelGGL(split_finish_kernel<T>, dim3((unsigned)ceil_div(len, 256)), dim3(256), 0, st, len,
                           nsplit, partial, out);
}

template <typename T>
static sb_status gemv_n_typed(sb_handle* h, int64_t rows, int64_t cols, const T* A, int64_t ld,
                              const T* x, T* c)
{
    const bool al = aligned16(A) && ((ld * (int64_t)sizeof(T)) % 16 == 0);
    const GemvNPlan p = plan_gemv_n(sizeof(T), rows, cols, !al);
    if (p.ws > h->ws_bytes)
        return fail(h, SB_ENOMEM, "gemv needs %zu workspace bytes, handle has %zu", p.ws, h->ws_bytes);
    if (p.nsplit > 65535)
        return fail(h, SB_EUNSUPPORTED, "gemv: rows of %lld elements need %lld column splits (at most 65535)",
                    (long long)cols, (long long)p.nsplit);
    GemvNArgs<T> a{rows, cols, ld, A, x, c, p.nsplit > 1 ? static_cast<T*>(claim_ws(h)) : nullptr, p.KC, p.RB};
    const dim3 grid((unsigned)ceil_div(rows, p.RB), (unsigned)p.nsplit);
    bool ok = true;
    if (p.pairs) {
        // binary32 rows not aligned, x read as 8-byte pairs from two copies
        if constexpr (std::is_same<T, float>::value) {
            if (p.lds > 80 * 1024 && p.NT == SB_GEMV_N_NT_HUGE && p.G == 64)
                launch_n<T, 64, SB_GEMV_N_NT_HUGE, false, kUnrollNHuge, false, true>(a, grid, p.lds, h->stream);
            else
                ok = dispatch_n<T, false, false, true>(p.NT, p.G, a, grid, p.lds, h->stream);
        } else {
            ok = false;
        }
    } else if (p.lds > 80 * 1024 && p.NT == SB_GEMV_N_NT_HUGE && p.G == 64) {
        // whole rows with x above 80 KiB: more loads in flight per lane
        if (al) launch_n<T, 64, SB_GEMV_N_NT_HUGE, true, kUnrollNHuge>(a, grid, p.lds, h->stream);
        else launch_n<T, 64, SB_GEMV_N_NT_HUGE, false, kUnrollNHuge>(a, grid, p.lds, h->stream);
    } else if (p.xcopies > 1) {
        ok = dispatch_n<T, false, true>(p.NT, p.G, a, grid, p.lds, h->stream);
    } else {
        ok = al ? dispatch_n<T, true>(p.NT, p.G, a, grid, p.lds, h->stream)
                : dispatch_n<T, false>(p.NT, p.G, a, grid, p.lds, h->stream);
    }
    if (!ok) return fail(h, SB_EINTERNAL, "no gemv_n instance for NT=%d G=%d", p.NT, p.G);
    sb_status st = check_launch(h, "gemv_n_kernel");
    if (st != SB_OK || p.nsplit == 1) return st;
    launch_split_finish<T>(h->stream, rows, p.nsplit, static_cast<const T*>(h->ws), c);
    return check_launch(h, "split_finish_kernel");
}

template <typename T>
static sb_status gemv_t_typed(sb_handle* h, int64_t rows, int64_t cols, const T* A, int64_t ld,
                              const T* x, T* c)
{
    const GemvTPlan p = plan_gemv_t(sizeof(T), rows, cols, h->gemv_t_small_splits);
    if (p.ws > h->ws_bytes)
        return fail(h, SB_ENOMEM, "gemv needs %zu workspace bytes, handle has %zu", p.ws, h->ws_bytes);
    GemvTArgs<T> a{rows, cols, ld, A, x, c, p.nsplit > 1 ? static_cast<T*>(claim_ws(h)) : nullptr, p.RS};
    const bool al = aligned16(A) && ((ld * (int64_t)sizeof(T)) % 16 == 0);
    const int64_t CW = 64 * (al ? 16 / (int64_t)sizeof(T) : 1);
    const dim3 grid((unsigned)ceil_div(cols, CW), (unsigned)p.nsplit);
    constexpr bool kPhaseForm = std::is_same<T, float>::value && SB_GEMV_T_PHASE;
    if (kPhaseForm && !al && p.NT == 256) {
        if constexpr (kPhaseForm)
            hipLaunchKernelGGL(gemv_t_phase_kernel<T>, dim3((unsigned)ceil_div(cols, 64 * 4), (unsigned)p.nsplit),
                               dim3(256), 0, h->stream, a);
    } else if (!al && p.NT == 256) {
        GemvTElemArgs<T> e{rows, cols, ld, A, x, c, a.partial, p.RS};
        hipLaunchKernelGGL(gemv_t_elem_kernel<T>, dim3((unsigned)ceil_div(cols, 256), (unsigned)p.nsplit), dim3(256),
                           0, h->stream, e);
    } else if (al && p.NT == 256 && p.nsplit == 1 && grid.x >= kGemvTBandBlocks && rows <= kGemvTBandRows) {
        hipLaunchKernelGGL(gemv_t_band_kernel<T>, dim3((unsigned)ceil_div(cols, 4 * CW)), dim3(256), 0, h->stream, a);
    } else if (p.NT == 1024) {
        if (al) hipLaunchKernelGGL((gemv_t_kernel<T, 1024, true>), grid, dim3(1024), 0, h->stream, a);
        else hipLaunchKernelGGL((gemv_t_kernel<T, 1024, false>), grid, dim3(1024), 0, h->stream, a);
    } else {
        if (al) hipLaunchKernelGGL((gemv_t_kernel<T, 256, true>), grid, dim3(256), 0, h->stream, a);
        else hipLaunchKernelGGL((gemv_t_kernel<T, 256, false>), grid, dim3(256), 0, h->stream, a);
    }
    sb_status st = check_launch(h, "gemv_t_kernel");
    if (st != SB_OK || p.nsplit == 1) return st;
    launch_split_finish<T>(h->stream, cols, p.nsplit, static_cast<const T*>(h->ws), c);
    return check_launch(h, "split_finish_kernel");
}

sb_status run_gemv_n(sb_handle* h, sb_dtype dt, int64_t rows, int64_t cols, const void* M,
                     int64_t ld, const void* v, void* out)
{
    if (rows == 0 || cols == 0) return SB_OK;
    if (dt == SB_F64)
        return gemv_n_typed<double>(h, rows, cols, static_cast<const double*>(M), ld,
                                    static_cast<const double*>(v), static_cast<double*>(out));
    return gemv_n_typed<float>(h, rows, cols, static_cast<const float*>(M), ld,
                               static_cast<const float*>(v), static_cast<float*>(out));
}

sb_status run_gemv_t(sb_handle* h, sb_dtype dt, int64_t rows, int64_t cols, const void* M,
                     int64_t ld, const void* v, void* out)
{
    if (rows == 0 || cols == 0) return SB_OK;
    if (dt == SB_F64)
        return gemv_t_typed<double>(h, rows, cols, static_cast<const double*>(M), ld,
                                    static_cast<const double*>(v), static_cast<double*>(out));
    return gemv_t_typed<float>(h, rows, cols, static_cast<const float*>(M), ld,
                               static_cast<const float*>(v), static_cast<float*>(out));
}

}  // namespace sb
