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
// A problem split into S column chunks writes per-split partial sums to
// scratch; the tile that completes a row tile (a per-row-tile counter
// reaches S) adds the partials in split order and then the initial c.  Every
// result therefore depends only on the problem and its (group, rows per
// tile, split) configuration, never on the rest of the batch or on which
// workgroup ran it: a problem gives the same bits alone and in a mix.
//
// The table (header, problem records, work items grouped by workgroup,
// zeroed split counters) is encoded on the host and copied to device memory
// before the launch; the kernel reads everything it needs from it, so a
// captured launch can be replayed over new tables written to the same
// address.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "sb_device.hpp"
#include "sb_internal.hpp"
#include "sb_rowdot.hpp"

namespace sb {

constexpr int kBatNT = 256;
constexpr int kBatWaves = kBatNT / kWave;
constexpr int64_t kBatLds = 32 * 1024;     // x chunk bytes per tile
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
// Cost of a tile for the division of the work: its bytes of A, a fixed
// SB_BAT_TILE_COST for the set-up and x staging, and SB_BAT_PASS_COST per row
// pass (one memory latency each).
#ifndef SB_BAT_TILE_COST
#define SB_BAT_TILE_COST 4096
#endif
#ifndef SB_BAT_PASS_COST
#define SB_BAT_PASS_COST 8192
#endif
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
#ifndef SB_BAT_GRID
#define SB_BAT_GRID 1024
#endif
constexpr int kBatUnrollPlain = SB_BAT_UNROLL_PLAIN, kBatUnrollBf16 = SB_BAT_UNROLL_BF16,
              kBatUnrollE4m3 = SB_BAT_UNROLL_E4M3;
// The items are dealt to 1024 workgroups, two rounds of the two that fit a
// compute unit: in the serving loop the operand generator runs beside the
// batched kernel, and finer lists let the batched workgroups fill whatever
// the generator leaves free (serving at 4e5 requests/s: 1.26e5 served per
// second against 1.10e5 with 512 lists); alone, 512 and 1024 lists run
// within noise of each other.
constexpr int kBatGrid = SB_BAT_GRID;

struct BatHeader {
    int64_t count;
    int64_t ntiles;
    int64_t total_cost;  // sum of tile costs, KiB units
    int64_t nitems;      // work items
    int64_t items_off;   // byte offset of the work items (grouped by workgroup)
    int64_t lists_off;   // byte offset of grid + 1 int32 offsets: workgroup b's items are [off[b], off[b + 1])
    int32_t grid;        // workgroups the items were dealt to
    int32_t pad;
    int64_t pad2;
};

struct BatProblem {
    int32_t dtype, G, RT, S;
    int64_t m, n, lda, KC;
    int64_t tile0, rtiles;
    int64_t cost0, tile_cost;  // cost before this problem's first tile, and per tile (KiB units)
    const void* A;
    const float* scales;
    const void* x;
    void* c;
    void* partial;
    int32_t* counters;
    int32_t aligned, pad;
    int64_t pad2;
};

// Tiles [first, first + count) (numbered within the problem) of one problem.
struct BatItem {
    int32_t problem;
    int32_t count;
    int64_t first;
};
static_assert(sizeof(BatHeader) == 64, "header layout");
static_assert(sizeof(BatProblem) == 144, "problem record layout");
static_assert(sizeof(BatItem) == 16, "work item layout");

// Rows [r0, r1) of one tile, per-row results to c or to the split partials.
// Inlined into the kernel, whose bound of two workgroups per compute unit
// leaves room for every (dtype, group, alignment) variant without spills
// (204 VGPRs): as separate non-inlined functions their call frames cost 160
// bytes of scratch per lane, and within 128 VGPRs the inlined variants spill.
template <int DT, int G, bool AL>
__device__ __forceinline__ void bat_rows(const BatProblem& p, int64_t s, int64_t r0, int64_t r1, int64_t k0,
                                         int64_t klen, const unsigned char* xs_raw)
{
    constexpr int GW = kWave / G;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int g = lane / G, l = lane % G;
    for (int64_t row = r0 + w * GW + g; row < r1; row += kBatWaves * GW) {
        if constexpr (DT == SB_F64 || DT == SB_F32) {
            typedef typename std::conditional<DT == SB_F64, double, float>::type T;
            const T* Ar = static_cast<const T*>(p.A) + row * p.lda + k0;
            T t = row_dot<T, G, kBatUnrollPlain, AL, true, false>(Ar, klen, reinterpret_cast<const T*>(xs_raw), l);
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
            tile_dot<C, G, U, 1, true, false>(static_cast<const code_t*>(p.A) + row * p.lda + k0, p.lda, klen,
                                       reinterpret_cast<const float*>(xs_raw), l, t);
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

// Second stage of a split row tile: c_i += (scale *) sum over splits in order.
template <typename T>
__device__ __forceinline__ void bat_finish(const BatProblem& p, int64_t r0, int64_t r1)
{
    const T* part = static_cast<const T*>(p.partial);
    T* c = static_cast<T*>(p.c);
    for (int64_t row = r0 + threadIdx.x; row < r1; row += kBatNT) {
        const T t = ordered_split_sum(part + row, (int64_t)p.S, p.m);
        if (p.dtype == SB_BF16 || p.dtype == SB_FP8_E4M3) c[row] = c[row] + p.scales[row] * t;
        else c[row] = c[row] + t;
    }
}

// Two workgroups per compute unit (two waves per SIMD).
__global__ __launch_bounds__(kBatNT, 2) void gemv_batched_kernel(const unsigned char* table)
{
    __shared__ __align__(16) unsigned char xs[kBatLds];
    __shared__ int last_flag;
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
            const int64_t s = local % p.S, rt = local / p.S;
            const int64_t r0 = rt * p.RT, r1 = min(p.m, r0 + p.RT);
            const int64_t k0 = s * p.KC, klen = min(p.n, k0 + p.KC) - k0;

            if (pi != cached_p || s != cached_s) {
                __syncthreads();  // every row of the previous tile has read x
                const int xs_size = p.dtype == SB_F64 ? 8 : 4;
                const unsigned char* xg = static_cast<const unsigned char*>(p.x) + k0 * xs_size;
                const int64_t nbytes = klen * xs_size;
                if (((reinterpret_cast<uintptr_t>(xg) | (uintptr_t)nbytes) & 15) == 0) {
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
            case SB_BF16: bat_rows_g<SB_BF16, false>(p, s, r0, r1, k0, klen, xs); break;
            default: bat_rows_g<SB_FP8_E4M3, false>(p, s, r0, r1, k0, klen, xs); break;
            }

            if (p.S > 1) {
                // Publish this split's partials; the tile that completes the
                // row tile adds all splits in order.
                __threadfence();
                __syncthreads();
                if (threadIdx.x == 0) {
                    last_flag = atomicAdd(&p.counters[rt], 1) == p.S - 1;
                    // every split of this row tile has arrived: rearm the
                    // counter so the same table can be launched again
                    if (last_flag) atomicExch(&p.counters[rt], 0);
                }
                __syncthreads();
                if (last_flag) {
                    __threadfence();
                    if (p.dtype == SB_F64) bat_finish<double>(p, r0, r1);
                    else bat_finish<float>(p, r0, r1);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ host ---

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

static int esize(int32_t dt) { return dt == SB_F64 ? 8 : dt == SB_F32 ? 4 : dt == SB_BF16 ? 2 : 1; }
static int xsize(int32_t dt) { return dt == SB_F64 ? 8 : 4; }

// Fill the automatic fields of one descriptor; false if it cannot be run.
static bool resolve(const sb_gemv_desc& in, sb_gemv_desc& out, int64_t* KC, int64_t tile_bytes, char* why,
                    size_t whylen)
{
    out = in;
    const int es = esize(in.dtype), xs = xsize(in.dtype);
    const int64_t vec = 16 / es;  // elements per 16-byte load
    const int64_t max_kc = kBatLds / xs;
    if (in.split < 0 || in.group < 0 || in.rows_per_tile < 0) {
        snprintf(why, whylen, "negative configuration value");
        return false;
    }
    int64_t S = in.split ? in.split : std::max<int64_t>(1, ceil_div(in.n, max_kc));
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

struct BatLayout {
    std::vector<sb_gemv_desc> res;
    std::vector<int64_t> kc, tiles, rtiles, tile_cost, counter_off, partial_off;
    std::vector<BatItem> items;
    int32_t grid = 0;            // workgroups the items are dealt to
    size_t image = 0, total = 0, items_off = 0, lists_off = 0;
    int64_t ntiles = 0, total_cost = 0;
};

static sb_status layout(const sb_gemv_desc* d, int32_t count, BatLayout& L, char* why, size_t whylen)
{
    if (count < 0 || (count > 0 && !d)) {
        snprintf(why, whylen, "bad descriptor array");
        return SB_EINVAL;
    }
    L.res.resize(count);
    L.kc.resize(count);
    L.tiles.resize(count);
    L.rtiles.resize(count);
    L.tile_cost.resize(count);
    L.counter_off.resize(count);
    L.partial_off.resize(count);
    // The rows of a tile never change a row's arithmetic, so results do not
    // depend on the tile size.
    const int64_t tile_bytes = kBatTileBytes;
    for (int32_t i = 0; i < count; ++i) {
        const sb_gemv_desc& in = d[i];
        if (in.dtype < SB_F64 || in.dtype > SB_FP8_E4M3 || in.m < 0 || in.n < 0 || in.lda < std::max<int64_t>(1, in.n)) {
            snprintf(why, whylen, "descriptor %d: bad dtype, size or lda", i);
            return SB_EINVAL;
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
        char sub[160];
        if (!resolve(in, L.res[i], &L.kc[i], tile_bytes, sub, sizeof sub)) {
            snprintf(why, whylen, "descriptor %d: %s", i, sub);
            return SB_EINVAL;
        }
        const sb_gemv_desc& r = L.res[i];
        const int64_t rt = (in.m == 0 || in.n == 0) ? 0 : ceil_div(in.m, r.rows_per_tile);
        L.rtiles[i] = rt;
        L.tiles[i] = rt * r.split;
        L.ntiles += L.tiles[i];
        // tile cost: its bytes of A, the set-up and x staging, and one
        // memory latency per row pass
        const int64_t a_bytes = (int64_t)r.rows_per_tile * std::min<int64_t>(L.kc[i], in.n) * es;
        const int64_t passes = ceil_div(r.rows_per_tile, (int64_t)kBatWaves * (64 / r.group));
        L.tile_cost[i] = L.tiles[i] > 0 ? (a_bytes + SB_BAT_TILE_COST + passes * SB_BAT_PASS_COST + 1023) / 1024 : 0;
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
    for (int32_t i = 0; i < count; ++i) {
        L.counter_off[i] = -1;
        if (L.res[i].split > 1 && L.rtiles[i] > 0) {
            L.counter_off[i] = (int64_t)off;
            off += (size_t)L.rtiles[i] * sizeof(int32_t);
        }
    }
    L.image = round_up((int64_t)off, 64);
    size_t total = L.image;
    for (int32_t i = 0; i < count; ++i) {
        L.partial_off[i] = -1;
        if (L.res[i].split > 1 && L.rtiles[i] > 0) {
            L.partial_off[i] = (int64_t)total;
            total += (size_t)round_up(L.res[i].split * d[i].m * xsize(d[i].dtype), 64);
        }
    }
    L.total = total;
    // Outputs of different problems must not overlap (each c has one owner).
    std::vector<std::pair<uintptr_t, uintptr_t>> cs;
    for (int32_t i = 0; i < count; ++i) {
        if (d[i].m > 0 && d[i].n > 0) {
            const uintptr_t lo = (uintptr_t)d[i].c;
            cs.push_back({lo, lo + (uintptr_t)d[i].m * xsize(d[i].dtype)});
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
        p.m = d[i].m;
        p.n = d[i].n;
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
        p.counters = L.counter_off[i] >= 0 ? reinterpret_cast<int32_t*>(dev_table + L.counter_off[i]) : nullptr;
        const int es = esize(r.dtype);
        p.aligned = (r.dtype == SB_F64 || r.dtype == SB_F32) && aligned16(d[i].A) && (d[i].lda * es) % 16 == 0;
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

sb_status sb_gemv_batched_run(sb_handle* handle, const void* dev_table, int32_t grid)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_gemv_batched_run: NULL handle");
    if (!dev_table || !sb::aligned16(dev_table)) return fail(handle, SB_EINVAL, "sb_gemv_batched_run: bad table");
    if (grid < 0 || grid > (1 << 20)) return fail(handle, SB_EINVAL, "sb_gemv_batched_run: bad grid %d", grid);
    const int g = grid ? grid : sb::kBatGrid;
    hipLaunchKernelGGL(sb::gemv_batched_kernel, dim3(g), dim3(sb::kBatNT), 0, handle->stream,
                       static_cast<const unsigned char*>(dev_table));
    return sb::check_launch(handle, "gemv_batched_kernel");
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
        return sb_gemv_batched_run(handle, handle->ws, 0);
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
        sb_plan* p = new (std::nothrow) sb_plan{handle, handle->ws, handle->ws_gen, L.ntiles};
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
    return sb_gemv_batched_run(h, plan->table, 0);
}

sb_status sb_plan_destroy(sb_plan* plan)
{
    delete plan;
    return SB_OK;
}

}  // extern "C"
