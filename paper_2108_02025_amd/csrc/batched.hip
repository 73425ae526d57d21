// Batched GEMV: many uneven problems c += A x in one persistent launch.
//
// The paper (section 4.2) observes that for small problems the cost of
// starting threads dominates and proposes fewer or no threads for them.  On
// the GPU the analogous fixed cost is a kernel launch, so a batch of
// problems shares one launch: every problem is cut into tiles of RT rows x KC
// columns (KC covering all of n unless the problem is split along its
// columns), and runs of consecutive tiles of one problem form work items.
// The host deals the items to the workgroups of a persistent grid, largest
// first, in rounds of one item per workgroup whose direction alternates
// (round 0 gives workgroup b the (b+1)-th largest item, round 1 the
// (2*grid-b)-th, and so on): no workgroup ends more than one item's cost
// above another, whatever the mix of shapes, and the device needs no
// counter traffic to share the work.
// A tile stages its x chunk in LDS (kept if the workgroup's next tile uses
// the same chunk) and runs the same per-row dot products as the single-call
// kernels.
//
// Both layouts and both operations are accepted (sections 4.1 and 4.2 treat
// both storage orders).  (row-major, N) and (column-major, T) are row dots
// over the stored rows, as above.  (row-major, T) and (column-major, N) are
// column axpys over the stored rows (the output runs along the stored
// columns): such a problem is cut into column blocks of one wave's width
// (64 lanes, each owning one 16-byte vector of consecutive columns, or one
// column if the rows are not 16-byte aligned) by row chunks; the four waves
// of the workgroup take alternate rows of a chunk, each lane adding its
// columns' products in row order, and the waves' sums are added in wave
// order through LDS.  Several row chunks write partial sums that the
// completing tile adds in chunk order, as for split row dots.
//
// A problem split into S column chunks writes per-split partial sums to
// scratch; a second kernel then adds each output's partials in split order
// and then the initial c.  (Handing the last split's tile the sum instead,
// through a counter, needs a device-scope release and acquire per tile,
// which on this chip write back and invalidate the whole L2 of the
// workgroup's XCD: binary64 8192^2 problems, all split in two, ran at
// 0.66 TB/s that way.)  Every result therefore depends only on the problem
// and its (group, rows per tile, split) configuration, never on the rest of
// the batch or on which workgroup ran it: a problem gives the same bits
// alone and in a mix.
//
// The table (header, problem records, work items grouped by workgroup, the
// second kernel's items) is encoded on the host and copied to device memory
// before the launch; the kernels read everything they need from it, so a
// captured launch can be replayed over new tables written to the same
// address.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "sb_device.hpp"
#include "sb_internal.hpp"
#include "sb_rowdot.hpp"

namespace sb {

constexpr int kBatNT = 256;
constexpr int kBatWaves = kBatNT / kWave;
// x chunk bytes per tile: two workgroups per compute unit, each with 64 KiB
// (68 KiB with the column-axpy buffer) of the 160 KiB of LDS
constexpr int64_t kBatLds = 64 * 1024;
// Code and binary32 rows that are not 16-byte aligned: two copies of x, copy h shifted
// left by h elements, kBatXStride elements apart, read as 8-byte pairs, so
// chunks of at most kBatXStride columns (the automatic or given split is
// raised to keep them so).
constexpr int64_t kBatXStride = kBatLds / 2 / 4;
// Automatic tile height: about SB_BAT_TILE_BYTES of A per tile, and at most
// SB_BAT_MAX_PASSES row passes of the workgroup (a pass: the rows its groups
// take at once), since short rows are latency-bound per pass.
#ifndef SB_BAT_TILE_BYTES
#define SB_BAT_TILE_BYTES (256 * 1024)
#endif
#ifndef SB_BAT_ITEMS_PER_WG
#define SB_BAT_ITEMS_PER_WG 8
#endif
#ifndef SB_BAT_MAX_PASSES
#define SB_BAT_MAX_PASSES 8
#endif
// Cost of a tile for the division of the work, in units of 10 ns: its
// bytes of A at a per-format rate, a latency per row pass (a pass waits for
// its loads) and a fixed part per tile.  The constants are a least-squares
// fit to the measured durations of 90k tiles of random batches (m, n
// log-uniform in [64, 8192], all four formats, tuned configurations):
// microseconds per MB of A 44.38 (binary64), 47.73 (binary32), 76.06
// (bfloat16 codes), 134.35 (E4M3 codes); 2.47 per pass; 0.37 per tile
// (R^2 0.84, against 0.43-0.58 for bytes + 4 KiB + 8 KiB per pass).
#ifndef SB_BAT_COST_PASS_US
#define SB_BAT_COST_PASS_US 2.47
#endif
#ifndef SB_BAT_COST_TILE_US
#define SB_BAT_COST_TILE_US 0.37
#endif
static double cost_us_per_mb(int32_t dt)
{
    return dt == SB_F64 ? 44.38 : dt == SB_F32 ? 47.73 : dt == SB_BF16 ? 76.06 : 134.35;
}
constexpr int64_t kBatTileBytes = SB_BAT_TILE_BYTES;  // largest automatic tile (bytes of A)
#ifndef SB_BAT_UNROLL_PLAIN
#define SB_BAT_UNROLL_PLAIN 8
#endif
#ifndef SB_BAT_UNROLL_BF16
#define SB_BAT_UNROLL_BF16 8
#endif
#ifndef SB_BAT_UNROLL_E4M3
#define SB_BAT_UNROLL_E4M3 4
#endif
#ifndef SB_BAT_UNROLL_T
#define SB_BAT_UNROLL_T 8
#endif
// The vectors of a row left after its full batches of U: one predicated
// batch, all in flight together (1), or one at a time (0), a round trip
// each.  The additions happen in the same order either way.
#ifndef SB_BAT_BATCH_TAIL
#define SB_BAT_BATCH_TAIL 1
#endif
#ifndef SB_BAT_GRID
#define SB_BAT_GRID 1024
#endif
constexpr int kBatUnrollPlain = SB_BAT_UNROLL_PLAIN, kBatUnrollBf16 = SB_BAT_UNROLL_BF16,
              kBatUnrollE4m3 = SB_BAT_UNROLL_E4M3;
constexpr int kBatUnrollT = SB_BAT_UNROLL_T;  // rows in flight per wave of a column-axpy tile (16-byte rows)
// The items are dealt to 1024 workgroups, two rounds of the two that fit a
// compute unit: in the serving loop the operand generator runs beside the
// batched kernel, and finer lists let the batched workgroups fill whatever
// the generator leaves free (serving at 4e5 requests/s: 1.26e5 served per
// second against 1.10e5 with 512 lists); alone, 512 and 1024 lists run
// within noise of each other.
constexpr int kBatGrid = SB_BAT_GRID;
constexpr int64_t kFinishChunk = 4 * kBatNT;  // outputs per second-stage item
constexpr int kFinishGrid = 256;              // second-stage workgroups

struct BatHeader {
    int64_t count;
    int64_t ntiles;
    int64_t total_cost;  // sum of tile costs, 10 ns units
    int64_t nitems;      // work items
    int64_t items_off;   // byte offset of the work items (grouped by workgroup)
    int64_t lists_off;   // byte offset of grid + 1 int32 offsets: workgroup b's items are [off[b], off[b + 1])
    int32_t grid;        // workgroups the items were dealt to
    int32_t nfinish;     // second-stage items (outputs of split problems, kFinishChunk at a time)
    int64_t finish_off;  // byte offset of the second-stage items
};

// m, n, lda describe the stored matrix: m stored rows of n contiguous
// elements.  Row dot (cols == 0): c has m entries, x n; RT rows per tile,
// KC columns per split.  Column axpy (cols == 1): c has n entries, x m; RT
// rows per chunk, KC columns per block; rtiles counts the output tiles (row
// tiles or column blocks).
struct BatProblem {
    int32_t dtype, G, RT, S;
    int64_t m, n, lda, KC;
    int64_t tile0, rtiles;
    int64_t cost0, tile_cost;  // cost before this problem's first tile, and per tile (10 ns units)
    const void* A;
    const float* scales;
    const void* x;
    void* c;
    void* partial;
    void* reserved;
    int32_t aligned, cols;
    int64_t pad2;
};

// Tiles [first, first + count) (numbered within the problem) of one problem;
// for the second stage, outputs [first, first + count).
struct BatItem {
    int32_t problem;
    int32_t count;
    int64_t first;
};
static_assert(sizeof(BatHeader) == 64, "header layout");
static_assert(sizeof(BatProblem) == 144, "problem record layout");
static_assert(sizeof(BatItem) == 16, "work item layout");
static_assert(sizeof(sb_gemv_desc) == 80, "descriptor layout (mirrored by the Python binding)");

// Rows [r0, r1) of one tile, per-row results to c or to the split partials.
// Inlined into the kernel, whose bound of two workgroups per compute unit
// leaves room for every (dtype, group, alignment) variant without spills
// (248 VGPRs): as separate non-inlined functions their call frames cost 160
// bytes of scratch per lane, and within 128 VGPRs the inlined variants spill.
template <int DT, int G, bool AL>
__device__ __forceinline__ void bat_rows(const BatProblem& p, int64_t s, int64_t r0, int64_t r1, int64_t k0,
                                         int64_t klen, const unsigned char* xs_raw)
{
    constexpr int GW = kWave / G;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int g = lane / G, l = lane % G;
    constexpr bool CODES = DT == SB_BF16 || DT == SB_FP8_E4M3;
    constexpr bool PHASED = CODES || (DT == SB_F32 && !AL);  // x read from copies
    // Rows that read x from the copies (codes; binary32 rows not 16-byte
    // aligned): the rows of one pass of a wave are `period` rows apart
    // (period: the rows after which the phase of a row start repeats; 1 for
    // aligned rows), so that its groups share the copy of x they read and
    // read the same addresses.  Pass slot q covers rows c + period (b GW + g),
    // c = q % period, b = q / period: every row of the tile once.  A row's
    // arithmetic does not depend on the order.
    int lp = 0;  // log2 of the period (a power of two, at most 16)
    if constexpr (PHASED) {
        const int rb = (int)((p.lda * (DT == SB_BF16 ? 2 : DT == SB_F32 ? 4 : 1)) & 15);
        lp = rb ? 4 - __builtin_ctz(rb) : 0;
    }
    const int64_t period = (int64_t)1 << lp;
    const int64_t nrows = r1 - r0;
    for (int64_t q = w;; q += kBatWaves) {
        int64_t row;
        if constexpr (PHASED) {
            const int64_t c = q & (period - 1), b = q >> lp;
            const int64_t base = c + period * b * GW;
            if (base >= nrows) break;
            row = r0 + base + period * g;
        } else {
            if (q * GW >= nrows) break;
            row = r0 + q * GW + g;
        }
        if (row >= r1) continue;
        if constexpr (DT == SB_F64 || DT == SB_F32) {
            typedef typename std::conditional<DT == SB_F64, double, float>::type T;
            const T* Ar = static_cast<const T*>(p.A) + row * p.lda + k0;
            // binary32 rows not aligned: x from copy head % 2 as 8-byte pairs
            constexpr bool PAIRS = DT == SB_F32 && !AL;
            T t = row_dot<T, G, kBatUnrollPlain, AL, true, SB_BAT_BATCH_TAIL, false, false, PAIRS>(
                Ar, klen, reinterpret_cast<const T*>(xs_raw), l, kBatXStride);
            t = group_sum<G>(t);
            if (l == 0) {
                if (p.S > 1) static_cast<T*>(p.partial)[s * p.m + row] = t;
                else static_cast<T*>(p.c)[row] = static_cast<T*>(p.c)[row] + t;
            }
        } else {
            typedef Codes<DT == SB_BF16> C;
            typedef typename C::code_t code_t;
            constexpr int U = DT == SB_BF16 ? kBatUnrollBf16 : kBatUnrollE4m3;
            float t[1];
            // x read as aligned vectors: 16 bytes from the single copy when
            // every row is 16-byte aligned (head 0), else 8-byte pairs from
            // copy head % 2
            const code_t* Qr = static_cast<const code_t*>(p.A) + row * p.lda + k0;
            const float* xf = reinterpret_cast<const float*>(xs_raw);
            if (p.aligned) tile_dot<C, G, U, 1, true, SB_BAT_BATCH_TAIL, false, 4>(Qr, p.lda, klen, xf, l, t, 0);
            else tile_dot<C, G, U, 1, true, SB_BAT_BATCH_TAIL, false, 2>(Qr, p.lda, klen, xf, l, t, kBatXStride);
            float v = group_sum<G>(t[0]);
            if (l == 0) {
                if (p.S > 1) static_cast<float*>(p.partial)[s * p.m + row] = v;
                else static_cast<float*>(p.c)[row] = static_cast<float*>(p.c)[row] + p.scales[row] * v;
            }
        }
    }
}

template <int DT, bool AL>
__device__ __forceinline__ void bat_rows_g(const BatProblem& p, int64_t s, int64_t r0, int64_t r1, int64_t k0,
                                           int64_t klen, const unsigned char* xs)
{
    switch (p.G) {
    case 4: bat_rows<DT, 4, AL>(p, s, r0, r1, k0, klen, xs); break;
    case 8: bat_rows<DT, 8, AL>(p, s, r0, r1, k0, klen, xs); break;
    case 16: bat_rows<DT, 16, AL>(p, s, r0, r1, k0, klen, xs); break;
    case 32: bat_rows<DT, 32, AL>(p, s, r0, r1, k0, klen, xs); break;
    default: bat_rows<DT, 64, AL>(p, s, r0, r1, k0, klen, xs); break;
    }
}

// Columns [j0, j1) of one row chunk of a column-axpy problem: c_j += sum_i
// A[i, j] x_i over the chunk's rows, or the chunk's partial sums.  red is
// 4 KiB of LDS.
template <typename T, bool AL>
__device__ __forceinline__ void bat_cols(const BatProblem& p, int64_t cb, int64_t s, unsigned char* red_raw)
{
    constexpr int W = AL ? Vec<T>::W : 1;
    typedef typename std::conditional<AL, typename Vec<T>::type, T>::type V;
    // rows in flight per wave: element loads move fewer bytes each
    constexpr int U = AL ? kBatUnrollT : 16 / (int)sizeof(T) * kBatUnrollT;
    constexpr int CW = kWave * W;
    static_assert(kBatWaves * CW * sizeof(T) <= 4096, "column-axpy LDS");
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t j0 = cb * CW + lane * W;
    const int64_t i0 = s * p.RT, i1 = min(p.m, i0 + p.RT);
    const T* A = static_cast<const T*>(p.A);
    const T* x = static_cast<const T*>(p.x);
    T acc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = 0;
    if (j0 + W <= p.n) {
        int64_t i = i0 + w;
        for (; i + (U - 1) * kBatWaves < i1; i += U * kBatWaves) {
            V av[U];
            T xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                av[u] = ld_stream<true>(reinterpret_cast<const V*>(A + (i + u * kBatWaves) * p.lda + j0));
                xv[u] = x[i + u * kBatWaves];
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
        for (; i < i1; i += kBatWaves) {
            const V av = ld_stream<true>(reinterpret_cast<const V*>(A + i * p.lda + j0));
            const T xv = x[i];
            if constexpr (W == 1) {
                acc[0] += av * xv;
            } else {
#pragma unroll
                for (int q = 0; q < W; ++q) acc[q] += av[q] * xv;
            }
        }
    } else if (j0 < p.n) {
        // right edge: fewer than W columns left for this lane
        const int rem = (int)(p.n - j0);
        for (int64_t i = i0 + w; i < i1; i += kBatWaves) {
            const T xv = x[i];
#pragma unroll
            for (int q = 0; q < W; ++q)
                if (q < rem) acc[q] += A[i * p.lda + j0 + q] * xv;
        }
    }
    T* red = reinterpret_cast<T*>(red_raw);
#pragma unroll
    for (int q = 0; q < W; ++q) red[w * CW + lane * W + q] = acc[q];
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int q = 0; q < W; ++q) {
            T t = red[lane * W + q];
#pragma unroll
            for (int k = 1; k < kBatWaves; ++k) t += red[k * CW + lane * W + q];
            const int64_t j = j0 + q;
            if (j < p.n) {
                if (p.S > 1) static_cast<T*>(p.partial)[s * p.n + j] = t;
                else static_cast<T*>(p.c)[j] = static_cast<T*>(p.c)[j] + t;
            }
        }
    }
    __syncthreads();  // red is written again by the next tile
}

// Two workgroups per compute unit (two waves per SIMD).
__global__ __launch_bounds__(kBatNT, 2) void gemv_batched_kernel(const unsigned char* table)
{
    __shared__ __align__(16) unsigned char xs[kBatLds];
    __shared__ __align__(16) unsigned char red[4096];
    const BatHeader* hdr = reinterpret_cast<const BatHeader*>(table);
    const BatProblem* probs = reinterpret_cast<const BatProblem*>(table + sizeof(BatHeader));
    const BatItem* items = reinterpret_cast<const BatItem*>(table + hdr->items_off);
    const int32_t* lists = reinterpret_cast<const int32_t*>(table + hdr->lists_off);
    const int64_t dealt = hdr->grid;
    int64_t cached_p = -1, cached_s = -1;

    // This workgroup's lists: its own, and those of workgroups beyond the
    // grid when the grid is smaller than the one the items were dealt to.
    for (int64_t b = blockIdx.x; b < dealt; b += gridDim.x)
    for (int64_t item = lists[b]; item < lists[b + 1]; ++item) {
        const BatItem it = items[item];
        const int64_t pi = it.problem;
        const BatProblem p = probs[pi];
        for (int64_t local = it.first; local < it.first + it.count; ++local) {
            // s: the split (column chunk of a row dot, row chunk of a column
            // axpy); rt: the output tile (row tile, or column block)
            const int64_t s = local % p.S, rt = local / p.S;
            const int64_t r0 = rt * p.RT, r1 = min(p.m, r0 + p.RT);
            const int64_t k0 = s * p.KC, klen = min(p.n, k0 + p.KC) - k0;

            if (p.cols) {
                if (p.dtype == SB_F64) {
                    if (p.aligned) bat_cols<double, true>(p, rt, s, red);
                    else bat_cols<double, false>(p, rt, s, red);
                } else {
                    if (p.aligned) bat_cols<float, true>(p, rt, s, red);
                    else bat_cols<float, false>(p, rt, s, red);
                }
            } else {
                if (pi != cached_p || s != cached_s) {
                    __syncthreads();  // every row of the previous tile has read x
                    const int xs_size = p.dtype == SB_F64 ? 8 : 4;
                    const unsigned char* xg = static_cast<const unsigned char*>(p.x) + k0 * xs_size;
                    const int64_t nbytes = klen * xs_size;
                    if ((p.dtype == SB_BF16 || p.dtype == SB_FP8_E4M3 || p.dtype == SB_F32) && !p.aligned) {
                        float* xf = reinterpret_cast<float*>(xs);
                        stage_to_lds<kBatNT, 16>(reinterpret_cast<const float*>(xg), klen, [&](int64_t e, float v) {
                            xf[e] = v;
                            if (e >= 1) xf[kBatXStride + e - 1] = v;
                        });
                    } else if (((reinterpret_cast<uintptr_t>(xg) | (uintptr_t)nbytes) & 15) == 0) {
                        stage_to_lds<kBatNT, 8>(reinterpret_cast<const v4u*>(xg), nbytes / 16,
                                                [&](int64_t e, v4u v) { reinterpret_cast<v4u*>(xs)[e] = v; });
                    } else {
                        stage_to_lds<kBatNT, 16>(reinterpret_cast<const uint32_t*>(xg), nbytes / 4,
                                                 [&](int64_t e, uint32_t v) { reinterpret_cast<uint32_t*>(xs)[e] = v; });
                    }
                    __syncthreads();
                    cached_p = pi;
                    cached_s = s;
                }

                switch (p.dtype) {
                case SB_F64:
                    if (p.aligned) bat_rows_g<SB_F64, true>(p, s, r0, r1, k0, klen, xs);
                    else bat_rows_g<SB_F64, false>(p, s, r0, r1, k0, klen, xs);
                    break;
                case SB_F32:
                    if (p.aligned) bat_rows_g<SB_F32, true>(p, s, r0, r1, k0, klen, xs);
                    else bat_rows_g<SB_F32, false>(p, s, r0, r1, k0, klen, xs);
                    break;
                // codes: one instance per format (alignment is a run-time
                // stride), which keeps the kernel's code small
                case SB_BF16: bat_rows_g<SB_BF16, false>(p, s, r0, r1, k0, klen, xs); break;
                default: bat_rows_g<SB_FP8_E4M3, false>(p, s, r0, r1, k0, klen, xs); break;
                }
            }
        }
    }
}

// Second stage: each item's outputs get the partial sums of their problem's
// splits added in split order, then the initial c (times the row's scale for
// codes).  Reads only the table, so it can follow any batched launch; a
// table without split problems has no items.
__global__ __launch_bounds__(kBatNT) void gemv_batched_finish_kernel(const unsigned char* table)
{
    const BatHeader* hdr = reinterpret_cast<const BatHeader*>(table);
    const BatProblem* probs = reinterpret_cast<const BatProblem*>(table + sizeof(BatHeader));
    const BatItem* fin = reinterpret_cast<const BatItem*>(table + hdr->finish_off);
    for (int64_t f = blockIdx.x; f < hdr->nfinish; f += gridDim.x) {
        const BatItem it = fin[f];
        const BatProblem& p = probs[it.problem];
        const int64_t stride = p.cols ? p.n : p.m;  // outputs of the problem
        for (int64_t o = it.first + threadIdx.x; o < it.first + it.count; o += kBatNT) {
            if (p.dtype == SB_F64) {
                double* c = static_cast<double*>(p.c);
                c[o] = c[o] + ordered_split_sum(static_cast<const double*>(p.partial) + o, (int64_t)p.S, stride);
            } else {
                float* c = static_cast<float*>(p.c);
                const float t = ordered_split_sum(static_cast<const float*>(p.partial) + o, (int64_t)p.S, stride);
                if (p.dtype == SB_BF16 || p.dtype == SB_FP8_E4M3) c[o] = c[o] + p.scales[o] * t;
                else c[o] = c[o] + t;
            }
        }
    }
}

// ------------------------------------------------------------------ host ---

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

static int esize(int32_t dt) { return dt == SB_F64 ? 8 : dt == SB_F32 ? 4 : dt == SB_BF16 ? 2 : 1; }
static int xsize(int32_t dt) { return dt == SB_F64 ? 8 : 4; }
// Stored rows that all start on a 16-byte boundary (binary64/32: 16-byte
// loads of whole rows; codes: x from the single copy as vectors).
static bool aligned_rows(int32_t dt, const void* A, int64_t lda)
{
    return aligned16(A) && (lda * esize(dt)) % 16 == 0;
}

// Fill the automatic fields of a row-dot descriptor (in.m, in.n: the stored
// rows and columns); false if it cannot be run.
static bool resolve_rows(const sb_gemv_desc& in, sb_gemv_desc& out, int64_t* KC, int64_t tile_bytes, char* why,
                         size_t whylen)
{
    out = in;
    const int es = esize(in.dtype), xs = xsize(in.dtype);
    const int64_t vec = 16 / es;  // elements per 16-byte load
    const bool codes = in.dtype == SB_BF16 || in.dtype == SB_FP8_E4M3;
    const bool shifted = (codes || in.dtype == SB_F32) && !aligned_rows(in.dtype, in.A, in.lda);  // two copies of x
    const int64_t max_kc = shifted ? kBatXStride : kBatLds / xs;
    if (in.split < 0 || in.group < 0 || in.rows_per_tile < 0) {
        snprintf(why, whylen, "negative configuration value");
        return false;
    }
    int64_t S = in.split ? in.split : std::max<int64_t>(1, ceil_div(in.n, max_kc));
    if (shifted) S = std::max<int64_t>(S, ceil_div(in.n, max_kc));
    int64_t kc = round_up(std::max<int64_t>(1, ceil_div(in.n, S)), 16);
    if (kc > max_kc) {
        snprintf(why, whylen, "split %lld leaves %lld columns per chunk, above %lld", (long long)S, (long long)kc,
                 (long long)max_kc);
        return false;
    }
    S = ceil_div(std::max<int64_t>(in.n, 1), kc);
    int G = in.group;
    if (G == 0) {
        const int U = in.dtype == SB_BF16 ? kBatUnrollBf16 : in.dtype == SB_FP8_E4M3 ? kBatUnrollE4m3 : kBatUnrollPlain;
        const int64_t nvec = ceil_div(kc, vec);
        G = 64;
        while (G > 4 && nvec < (int64_t)G * U) G >>= 1;
    } else if (G != 4 && G != 8 && G != 16 && G != 32 && G != 64) {
        snprintf(why, whylen, "group %d is not 4, 8, 16, 32 or 64", G);
        return false;
    }
    const int64_t pass = (int64_t)kBatWaves * (64 / G);
    int64_t RT = in.rows_per_tile;
    if (RT == 0) {
        const int64_t row_bytes = std::max<int64_t>(1, std::min<int64_t>(kc, in.n)) * es;
        RT = std::max<int64_t>(pass, (tile_bytes / row_bytes) / pass * pass);
        RT = std::min<int64_t>(RT, (int64_t)SB_BAT_MAX_PASSES * pass);
        RT = std::min<int64_t>(RT, round_up(std::max<int64_t>(in.m, 1), pass));
    } else if (RT % pass) {
        snprintf(why, whylen, "rows_per_tile %lld is not a multiple of %lld", (long long)RT, (long long)pass);
        return false;
    }
    if (RT > (1 << 30)) RT = 1 << 30;
    out.group = G;
    out.rows_per_tile = (int32_t)RT;
    out.split = (int32_t)S;
    *KC = kc;
    return true;
}

// The same for a column-axpy descriptor (in.m stored rows of in.n columns):
// rows_per_tile is the row chunk of a tile and split the number of chunks
// (either may be given; 0 for both: about tile_bytes of A per tile).  *CW
// receives the column block width.  group does not apply (0).
static bool resolve_cols(const sb_gemv_desc& in, bool aligned, sb_gemv_desc& out, int64_t* CW, int64_t tile_bytes,
                         char* why, size_t whylen)
{
    out = in;
    if (in.split < 0 || in.group < 0 || in.rows_per_tile < 0) {
        snprintf(why, whylen, "negative configuration value");
        return false;
    }
    if (in.group != 0) {
        snprintf(why, whylen, "group applies to row dots (row-major N, column-major T), not to column axpys");
        return false;
    }
    const int es = esize(in.dtype);
    const int64_t cw = (int64_t)kWave * (aligned ? 16 / es : 1);
    const int64_t pass = (int64_t)kBatWaves * (aligned ? kBatUnrollT : 16 / es * kBatUnrollT);
    const int64_t rows = std::max<int64_t>(in.m, 1);
    int64_t RT = in.rows_per_tile;
    if (RT == 0 && in.split > 0) {
        RT = ceil_div(rows, in.split);
    } else if (RT == 0) {
        const int64_t row_bytes = std::min<int64_t>(cw, std::max<int64_t>(in.n, 1)) * es;
        RT = std::max<int64_t>(pass, (tile_bytes / row_bytes) / pass * pass);
        RT = std::min<int64_t>(RT, round_up(rows, pass));
    }
    if (RT > (1 << 30)) RT = 1 << 30;
    const int64_t S = ceil_div(rows, RT);
    if (in.rows_per_tile > 0 && in.split > 0 && in.split != S) {
        snprintf(why, whylen, "split %d and rows_per_tile %d disagree (%lld chunks)", in.split, in.rows_per_tile,
                 (long long)S);
        return false;
    }
    if (S > (1 << 30)) {
        snprintf(why, whylen, "too many row chunks");
        return false;
    }
    out.group = 0;
    out.rows_per_tile = (int32_t)RT;
    out.split = (int32_t)S;
    *CW = cw;
    return true;
}

struct BatLayout {
    std::vector<sb_gemv_desc> res;  // the descriptors with their configuration resolved
    std::vector<int64_t> rows, cols;  // the stored matrix
    std::vector<int32_t> colform;     // 1: column axpy over the stored rows, 0: row dot
    std::vector<int64_t> kc, tiles, rtiles, tile_cost, partial_off;
    std::vector<BatItem> items;
    std::vector<BatItem> finish;  // second-stage items
    int32_t grid = 0;            // workgroups the items are dealt to
    size_t image = 0, total = 0, items_off = 0, lists_off = 0, finish_off = 0;
    int64_t ntiles = 0, total_cost = 0;
};

static sb_status layout(const sb_gemv_desc* d, int32_t count, BatLayout& L, char* why, size_t whylen)
{
    if (count < 0 || (count > 0 && !d)) {
        snprintf(why, whylen, "bad descriptor array");
        return SB_EINVAL;
    }
    L.res.resize(count);
    L.rows.resize(count);
    L.cols.resize(count);
    L.colform.resize(count);
    L.kc.resize(count);
    L.tiles.resize(count);
    L.rtiles.resize(count);
    L.tile_cost.resize(count);
    L.partial_off.resize(count);
    // The rows of a tile never change a row's arithmetic, so results do not
    // depend on the tile size.
    const int64_t tile_bytes = kBatTileBytes;
    for (int32_t i = 0; i < count; ++i) {
        const sb_gemv_desc& in = d[i];
        if ((in.layout != SB_ROW_MAJOR && in.layout != SB_COL_MAJOR) || (in.op != SB_N && in.op != SB_T)) {
            snprintf(why, whylen, "descriptor %d: bad layout or op", i);
            return SB_EINVAL;
        }
        const bool colmajor = in.layout == SB_COL_MAJOR;
        const int64_t rows = colmajor ? in.n : in.m, cols = colmajor ? in.m : in.n;
        if (in.dtype < SB_F64 || in.dtype > SB_FP8_E4M3 || in.m < 0 || in.n < 0 || in.lda < std::max<int64_t>(1, cols)) {
            snprintf(why, whylen, "descriptor %d: bad dtype, size or lda", i);
            return SB_EINVAL;
        }
        if ((in.dtype == SB_BF16 || in.dtype == SB_FP8_E4M3) && (colmajor || in.op != SB_N)) {
            snprintf(why, whylen, "descriptor %d: quantised problems are row-major N (the scales belong to rows)", i);
            return SB_EUNSUPPORTED;
        }
        if (in.m > 0 && in.n > 0 && (!in.A || !in.x || !in.c ||
                                     ((in.dtype == SB_BF16 || in.dtype == SB_FP8_E4M3) && !in.scales))) {
            snprintf(why, whylen, "descriptor %d: NULL pointer", i);
            return SB_EINVAL;
        }
        const int es = esize(in.dtype), xs = xsize(in.dtype);
        if ((uintptr_t)in.A % es || (uintptr_t)in.x % xs || (uintptr_t)in.c % xs || (uintptr_t)in.scales % 4) {
            snprintf(why, whylen, "descriptor %d: misaligned pointer", i);
            return SB_EINVAL;
        }
        if (in.m > (int64_t)1 << 40 || in.n > (int64_t)1 << 40 || in.lda > (int64_t)1 << 40) {
            snprintf(why, whylen, "descriptor %d: size too large", i);
            return SB_EINVAL;
        }
        // row-major N and column-major T are row dots over the stored rows;
        // row-major T and column-major N are column axpys over them
        const bool colform = colmajor == (in.op == SB_N);
        L.rows[i] = rows;
        L.cols[i] = cols;
        L.colform[i] = colform;
        sb_gemv_desc st = in;  // the stored form
        st.m = rows;
        st.n = cols;
        const bool al = aligned_rows(in.dtype, in.A, in.lda);
        char sub[160];
        if (!(colform ? resolve_cols(st, al, L.res[i], &L.kc[i], tile_bytes, sub, sizeof sub)
                      : resolve_rows(st, L.res[i], &L.kc[i], tile_bytes, sub, sizeof sub))) {
            snprintf(why, whylen, "descriptor %d: %s", i, sub);
            return SB_EINVAL;
        }
        L.res[i].m = in.m;
        L.res[i].n = in.n;
        const sb_gemv_desc& r = L.res[i];
        // output tiles: row tiles of a row dot, column blocks of a column axpy
        const int64_t rt = (rows == 0 || cols == 0) ? 0 : colform ? ceil_div(cols, L.kc[i]) : ceil_div(rows, r.rows_per_tile);
        L.rtiles[i] = rt;
        L.tiles[i] = rt * r.split;
        L.ntiles += L.tiles[i];
        // tile cost: its bytes of A, the set-up and x staging, and one
        // memory latency per row pass
        const int64_t a_bytes = (int64_t)r.rows_per_tile * std::min<int64_t>(L.kc[i], cols) * es;
        const int64_t pass = colform ? (int64_t)kBatWaves * (al ? kBatUnrollT : 16 / es * kBatUnrollT)
                                     : (int64_t)kBatWaves * (64 / r.group);
        const int64_t passes = ceil_div(r.rows_per_tile, pass);
        L.tile_cost[i] = L.tiles[i] > 0
                             ? std::max<int64_t>(1, std::llround(100.0 * (cost_us_per_mb(in.dtype) * 1e-6 * (double)a_bytes +
                                                                          SB_BAT_COST_PASS_US * (double)passes +
                                                                          SB_BAT_COST_TILE_US)))
                             : 0;
        L.total_cost += L.tile_cost[i] * L.tiles[i];
    }
    // Work items: runs of consecutive tiles of one problem costing about
    // 1/SB_BAT_ITEMS_PER_WG of a workgroup's share of the batch, listed in
    // problem and tile order (dealt to the workgroups by deal_items).
    const int64_t target = std::max<int64_t>(1, L.total_cost / ((int64_t)SB_BAT_ITEMS_PER_WG * kBatGrid));
    for (int32_t i = 0; i < count; ++i) {
        if (L.tiles[i] == 0) continue;
        const int64_t per =
            std::min<int64_t>(std::max<int64_t>(1, (target + L.tile_cost[i] / 2) / L.tile_cost[i]), (int64_t)1 << 30);
        for (int64_t first = 0; first < L.tiles[i]; first += per)
            L.items.push_back(BatItem{i, (int32_t)std::min<int64_t>(per, L.tiles[i] - first), first});
        if (L.items.size() > ((size_t)1 << 30)) {
            snprintf(why, whylen, "too many work items");
            return SB_EINVAL;
        }
    }
    L.grid = kBatGrid;
    size_t off = sizeof(BatHeader) + (size_t)count * sizeof(BatProblem);
    L.items_off = off;
    off += L.items.size() * sizeof(BatItem);
    L.lists_off = off;
    off += (size_t)(L.grid + 1) * sizeof(int32_t);
    // second stage: the outputs of every split problem, in chunks
    for (int32_t i = 0; i < count; ++i) {
        if (L.res[i].split <= 1 || L.rtiles[i] == 0) continue;
        const int64_t out_len = L.colform[i] ? L.cols[i] : L.rows[i];
        for (int64_t first = 0; first < out_len; first += kFinishChunk)
            L.finish.push_back(BatItem{i, (int32_t)std::min<int64_t>(kFinishChunk, out_len - first), first});
        if (L.finish.size() > ((size_t)1 << 30)) {
            snprintf(why, whylen, "too many outputs");
            return SB_EINVAL;
        }
    }
    L.finish_off = off;
    off += L.finish.size() * sizeof(BatItem);
    L.image = round_up((int64_t)off, 64);
    size_t total = L.image;
    for (int32_t i = 0; i < count; ++i) {
        L.partial_off[i] = -1;
        if (L.res[i].split > 1 && L.rtiles[i] > 0) {
            L.partial_off[i] = (int64_t)total;
            const int64_t out_len = L.colform[i] ? L.cols[i] : L.rows[i];
            total += (size_t)round_up(L.res[i].split * out_len * xsize(d[i].dtype), 64);
        }
    }
    L.total = total;
    // Outputs of different problems must not overlap (each c has one owner).
    std::vector<std::pair<uintptr_t, uintptr_t>> cs;
    for (int32_t i = 0; i < count; ++i) {
        if (d[i].m > 0 && d[i].n > 0) {
            const uintptr_t lo = (uintptr_t)d[i].c;
            const int64_t out_len = L.colform[i] ? L.cols[i] : L.rows[i];
            cs.push_back({lo, lo + (uintptr_t)out_len * xsize(d[i].dtype)});
        }
    }
    std::sort(cs.begin(), cs.end());
    for (size_t k = 1; k < cs.size(); ++k) {
        if (cs[k].first < cs[k - 1].second) {
            snprintf(why, whylen, "outputs of two problems overlap");
            return SB_EINVAL;
        }
    }
    return SB_OK;
}

// Deal the work items (in problem and tile order in L.items) to the
// workgroups, largest first (close to the longest-processing-time-first
// rule, in linear time after sorting at most two runs per problem).
// Writes the items grouped by workgroup, each group still in problem and
// tile order (so consecutive tiles of one problem reuse the staged x), and
// the grid + 1 group offsets.
static void deal_items(const BatLayout& L, BatItem* out, int32_t* lists)
{
    const size_t n = L.items.size();
    const int32_t grid = L.grid;
    if (n <= (size_t)grid) {  // one item per workgroup: nothing to balance
        for (size_t j = 0; j < n; ++j) out[j] = L.items[j];
        for (int32_t b = 0; b <= grid; ++b) lists[b] = (int32_t)std::min<size_t>((size_t)b, n);
        return;
    }
    // The items in (-cost, index) order (largest first, ties in item order).
    // A problem's items are consecutive and cost the same except its last
    // one, so that order is a sequence of runs of consecutive items: sort the
    // runs by (-cost, first index) rather than the items themselves (runs of
    // equal cost cover disjoint index ranges, so the order is the same).
    struct Run {
        int64_t neg_cost;
        size_t first, len;
    };
    std::vector<Run> runs;
    for (size_t j = 0; j < n;) {
        const int32_t p = L.items[j].problem;
        const int64_t c = L.items[j].count * L.tile_cost[p];
        size_t k = j + 1;
        while (k < n && L.items[k].problem == p && L.items[k].count * L.tile_cost[p] == c) ++k;
        runs.push_back(Run{-c, j, k - j});
        j = k;
    }
    std::sort(runs.begin(), runs.end(), [](const Run& a, const Run& b) {
        return a.neg_cost != b.neg_cost ? a.neg_cost < b.neg_cost : a.first < b.first;
    });
    std::vector<uint32_t> order(n);
    size_t at = 0;
    for (const Run& r : runs)
        for (size_t j = r.first; j < r.first + r.len; ++j) order[at++] = (uint32_t)j;
    // Largest first in rounds of `grid` items, alternating direction (the
    // snake order): round 0 gives workgroup b the (b+1)-th largest item,
    // round 1 pairs it with the (2*grid-b)-th, and so on, so each round
    // evens out the previous one; no workgroup ends above another by more
    // than the largest item.
    std::vector<int32_t> owner(n);
    for (size_t k = 0; k < n; ++k) {
        const size_t r = k / (size_t)grid, pos = k % (size_t)grid;
        owner[order[k]] = (int32_t)((r & 1) ? (size_t)grid - 1 - pos : pos);
    }
    std::vector<int32_t> fill(grid + 1, 0);
    for (size_t j = 0; j < n; ++j) ++fill[owner[j] + 1];
    for (int32_t b = 0; b < grid; ++b) fill[b + 1] += fill[b];
    for (int32_t b = 0; b <= grid; ++b) lists[b] = fill[b];
    for (size_t j = 0; j < n; ++j) out[fill[owner[j]]++] = L.items[j];  // creation order within a group
}

static void encode(const sb_gemv_desc* d, int32_t count, const BatLayout& L, unsigned char* dev_table,
                   unsigned char* image)
{
    memset(image, 0, L.image);
    BatHeader* hdr = reinterpret_cast<BatHeader*>(image);
    hdr->count = count;
    hdr->ntiles = L.ntiles;
    hdr->nitems = (int64_t)L.items.size();
    hdr->items_off = (int64_t)L.items_off;
    hdr->lists_off = (int64_t)L.lists_off;
    hdr->grid = L.grid;
    hdr->nfinish = (int32_t)L.finish.size();
    hdr->finish_off = (int64_t)L.finish_off;
    if (!L.finish.empty()) memcpy(image + L.finish_off, L.finish.data(), L.finish.size() * sizeof(BatItem));
    deal_items(L, reinterpret_cast<BatItem*>(image + L.items_off), reinterpret_cast<int32_t*>(image + L.lists_off));
    BatProblem* P = reinterpret_cast<BatProblem*>(image + sizeof(BatHeader));
    int64_t tile0 = 0, cost = 0;
    for (int32_t i = 0; i < count; ++i) {
        const sb_gemv_desc& r = L.res[i];
        BatProblem& p = P[i];
        p.dtype = r.dtype;
        p.G = r.group;
        p.RT = r.rows_per_tile;
        p.S = r.split;
        p.m = L.rows[i];
        p.n = L.cols[i];
        p.lda = d[i].lda;
        p.KC = L.kc[i];
        p.tile0 = tile0;
        p.rtiles = L.rtiles[i];
        p.tile_cost = L.tile_cost[i];
        p.cost0 = cost;
        cost += p.tile_cost * L.tiles[i];
        p.A = d[i].A;
        p.scales = d[i].scales;
        p.x = d[i].x;
        p.c = d[i].c;
        p.partial = L.partial_off[i] >= 0 ? dev_table + L.partial_off[i] : nullptr;
        p.aligned = aligned_rows(r.dtype, d[i].A, d[i].lda);
        p.cols = L.colform[i];
        tile0 += L.tiles[i];
    }
    hdr->total_cost = cost;
}

}  // namespace sb

using sb::fail;

extern "C" {

size_t sb_gemv_batched_table_bytes(const sb_gemv_desc* descs, int32_t count, size_t* image_bytes)
{
    sb::BatLayout L;
    char why[256];
    if (sb::layout(descs, count, L, why, sizeof why) != SB_OK) return (size_t)-1;
    if (image_bytes) *image_bytes = L.image;
    return L.total;
}

sb_status sb_gemv_batched_resolve(const sb_gemv_desc* descs, int32_t count, sb_gemv_desc* out)
{
    sb::BatLayout L;
    char why[256];
    if (!out && count > 0) return fail(nullptr, SB_EINVAL, "sb_gemv_batched_resolve: NULL output");
    const sb_status st = sb::layout(descs, count, L, why, sizeof why);
    if (st != SB_OK) return fail(nullptr, st, "sb_gemv_batched_resolve: %s", why);
    for (int32_t i = 0; i < count; ++i) out[i] = L.res[i];
    return SB_OK;
}

sb_status sb_gemv_batched_encode(const sb_gemv_desc* descs, int32_t count, void* dev_table, void* host_image,
                                 size_t image_bytes)
{
    sb::BatLayout L;
    char why[256];
    const sb_status st = sb::layout(descs, count, L, why, sizeof why);
    if (st != SB_OK) return fail(nullptr, st, "sb_gemv_batched_encode: %s", why);
    if (!dev_table || !host_image || image_bytes < L.image || !sb::aligned16(dev_table))
        return fail(nullptr, SB_EINVAL, "sb_gemv_batched_encode: table buffers missing, misaligned or too small");
    sb::encode(descs, count, L, static_cast<unsigned char*>(dev_table), static_cast<unsigned char*>(host_image));
    return SB_OK;
}

namespace sb {
// The persistent kernel, then (finish_grid > 0) the second stage.
static sb_status launch_batched(sb_handle* h, const void* dev_table, int grid, int finish_grid)
{
    hipLaunchKernelGGL(gemv_batched_kernel, dim3(grid), dim3(kBatNT), 0, h->stream,
                       static_cast<const unsigned char*>(dev_table));
    const sb_status st = check_launch(h, "gemv_batched_kernel");
    if (st != SB_OK || finish_grid == 0) return st;
    hipLaunchKernelGGL(gemv_batched_finish_kernel, dim3(finish_grid), dim3(kBatNT), 0, h->stream,
                       static_cast<const unsigned char*>(dev_table));
    return check_launch(h, "gemv_batched_finish_kernel");
}
static int finish_grid(size_t nfinish) { return (int)std::min<size_t>(nfinish, (size_t)kFinishGrid); }
}  // namespace sb

sb_status sb_gemv_batched_run(sb_handle* handle, const void* dev_table, int32_t grid)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_gemv_batched_run: NULL handle");
    if (!dev_table || !sb::aligned16(dev_table)) return fail(handle, SB_EINVAL, "sb_gemv_batched_run: bad table");
    if (grid < 0 || grid > (1 << 20)) return fail(handle, SB_EINVAL, "sb_gemv_batched_run: bad grid %d", grid);
    // The table may be rewritten between replays of a captured run, so the
    // second stage is always launched (it returns at once without items).
    return sb::launch_batched(handle, dev_table, grid ? grid : sb::kBatGrid, sb::kFinishGrid);
}

sb_status sb_gemv_batched(sb_handle* handle, const sb_gemv_desc* descs, int32_t count)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_gemv_batched: NULL handle");
    try {
        sb::BatLayout L;
        char why[256];
        const sb_status st = sb::layout(descs, count, L, why, sizeof why);
        if (st != SB_OK) return fail(handle, st, "sb_gemv_batched: %s", why);
        if (L.ntiles == 0) return SB_OK;
        if (L.total > handle->ws_bytes || !sb::aligned16(handle->ws))
            return fail(handle, SB_ENOMEM, "sb_gemv_batched needs %zu workspace bytes, handle has %zu", L.total,
                        handle->ws_bytes);
        std::vector<unsigned char> image(L.image);
        sb::encode(descs, count, L, static_cast<unsigned char*>(sb::claim_ws(handle)), image.data());
        // From pageable memory the copy is staged before the call returns,
        // so the local image may be released afterwards.
        const hipError_t e = hipMemcpyAsync(handle->ws, image.data(), L.image, hipMemcpyHostToDevice, handle->stream);
        if (e != hipSuccess) return fail(handle, SB_EDEVICE, "sb_gemv_batched: copy of the table: %s", hipGetErrorString(e));
        return sb::launch_batched(handle, handle->ws, sb::kBatGrid, sb::finish_grid(L.finish.size()));
    } catch (...) {
        return fail(handle, SB_EINTERNAL, "sb_gemv_batched: unexpected C++ exception");
    }
}

}  // extern "C"

// A batched plan: the table encoded once into the handle's workspace, run
// any number of times without host work.
struct sb_plan {
    sb_handle* handle;
    void* table;
    uint64_t gen;
    int64_t ntiles;
    int finish_grid;  // second-stage workgroups (0: no split problem)
};

extern "C" {

sb_status sb_plan_create(sb_handle* handle, const sb_gemv_desc* descs, int32_t count, sb_plan** out)
{
    if (!out) return fail(handle, SB_EINVAL, "sb_plan_create: out is NULL");
    *out = nullptr;
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_plan_create: NULL handle");
    try {
        sb::BatLayout L;
        char why[256];
        const sb_status st = sb::layout(descs, count, L, why, sizeof why);
        if (st != SB_OK) return fail(handle, st, "sb_plan_create: %s", why);
        if (L.ntiles > 0) {
            if (L.total > handle->ws_bytes || !sb::aligned16(handle->ws))
                return fail(handle, SB_ENOMEM, "sb_plan_create needs %zu workspace bytes, handle has %zu", L.total,
                            handle->ws_bytes);
            std::vector<unsigned char> image(L.image);
            sb::encode(descs, count, L, static_cast<unsigned char*>(sb::claim_ws(handle)), image.data());
            const hipError_t e =
                hipMemcpyAsync(handle->ws, image.data(), L.image, hipMemcpyHostToDevice, handle->stream);
            if (e != hipSuccess)
                return fail(handle, SB_EDEVICE, "sb_plan_create: copy of the table: %s", hipGetErrorString(e));
        }
        sb_plan* p = new (std::nothrow) sb_plan{handle, handle->ws, handle->ws_gen, L.ntiles,
                                                sb::finish_grid(L.finish.size())};
        if (!p) return fail(handle, SB_EINTERNAL, "sb_plan_create: out of host memory");
        *out = p;
        return SB_OK;
    } catch (...) {
        return fail(handle, SB_EINTERNAL, "sb_plan_create: unexpected C++ exception");
    }
}

sb_status sb_plan_run(sb_plan* plan)
{
    if (!plan) return fail(nullptr, SB_EINVAL, "sb_plan_run: NULL plan");
    if (plan->ntiles == 0) return SB_OK;
    sb_handle* h = plan->handle;
    if (h->ws != plan->table || h->ws_gen != plan->gen)
        return fail(h, SB_EINVAL, "sb_plan_run: the handle's workspace was replaced or written by a later call; "
                                  "create the plan again");
    return sb::launch_batched(h, plan->table, sb::kBatGrid, plan->finish_grid);
}

sb_status sb_plan_destroy(sb_plan* plan)
{
    delete plan;
    return SB_OK;
}

}  // extern "C"
