// On-device operand generation for the serving loop: counter-based uniform
// values in [-1, 1) from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).
// Element k of a fill is generated from counter c = counter0 + k:
//   z = seed + (c + 1) * 0x9E3779B97F4A7C15
//   z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
//   z = (z ^ (z >> 27)) * 0x94D049BB133111EB
//   z =  z ^ (z >> 31)
//   binary64: u = (z >> 11) * 2^-53 in [0, 1), value = 2u - 1 (exact)
//   binary32: two values per state: element e uses the state of counter
//     e >> 1 and the 24-bit field f = z >> 40 (e even) or (z >> 8) & 0xFFFFFF
//     (e odd); value = (f - 2^23) * 2^-23 (exact)
// The binary32 form needs no binary64 arithmetic and half the hashing per
// value, which made the operand generator about twice as fast.  Generating
// operands where they are used
// keeps host-to-device copies off the request path; any element can be
// regenerated on its own from (seed, counter).
#include <algorithm>

#include <string.h>

#include <vector>

#include "sb_device.hpp"
#include "sb_internal.hpp"
#include "sb_quant.hpp"

namespace sb {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

// The output of a SplitMix64 state z = seed + (c + 1) * golden (mod 2^64).
__device__ __forceinline__ double splitmix_from_state(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    const double u = (double)(z >> 11) * 0x1.0p-53;
    return 2.0 * u - 1.0;
}

// The two binary32 outputs of a state (elements 2c and 2c + 1).
__device__ __forceinline__ void splitmix_f32_pair(uint64_t z, float& even, float& odd)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    even = (float)((int32_t)(uint32_t)(z >> 40) - (1 << 23)) * 0x1.0p-23f;
    odd = (float)((int32_t)((uint32_t)(z >> 8) & 0xFFFFFFu) - (1 << 23)) * 0x1.0p-23f;
}

// Counters c, c + stride, c + 2 * stride, ...: the state advances by
// stride * golden each step (one addition instead of a multiplication).
struct SplitMixWalk {
    uint64_t z, step;
    __device__ SplitMixWalk(uint64_t seed, uint64_t c, uint64_t stride)
        : z(seed + (c + 1ull) * kGolden), step(stride * kGolden) {}
    __device__ double next()
    {
        const double v = splitmix_from_state(z);
        z += step;
        return v;
    }
    __device__ void next_f32_pair(float& even, float& odd)
    {
        splitmix_f32_pair(z, even, odd);
        z += step;
    }
};

// Elements [e0, e0 + len) of a stream taken in pairs (2p, 2p + 1) by lane l
// of a group of L lanes: pairs p = e0/2 + l, e0/2 + l + L, ..., up to the
// pair of the last element; visit(p, j) gets each pair with j = 2p - e0, the
// range index of its even element (-1 when the range starts on an odd
// element; j + 1 may be len when it ends on an even one).  Nothing is
// visited for an empty range.
template <int L, typename F>
__device__ __forceinline__ void for_pairs(uint64_t e0, int64_t len, int l, F visit)
{
    if (len <= 0) return;
    const uint64_t p0 = e0 >> 1, p1 = (e0 + (uint64_t)len - 1) >> 1;
    for (uint64_t p = p0 + (uint64_t)l; p <= p1; p += L) visit(p, (int64_t)(2 * p - e0));
}

// Binary32 elements [e0, e0 + len) of a counter stream, lane l of a group of
// L lanes: put(j, value) for each element j - e0 of the lane's pairs that
// lies inside the range.
template <int L, typename F>
__device__ __forceinline__ void f32_stream(uint64_t seed, uint64_t e0, int64_t len, int l, F put)
{
    SplitMixWalk g(seed, (e0 >> 1) + (uint64_t)l, L);
    for_pairs<L>(e0, len, l, [&](uint64_t, int64_t j) {
        float v0, v1;
        g.next_f32_pair(v0, v1);
        if (j >= 0) put(j, v0);
        if (j + 1 < len) put(j + 1, v1);
    });
}

__global__ __launch_bounds__(256) void fill_uniform_f64_kernel(double* out, int64_t count, uint64_t seed,
                                                               uint64_t counter0)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    SplitMixWalk g(seed, counter0 + (uint64_t)k, (uint64_t)stride);
    for (; k < count; k += stride) out[k] = g.next();
}

// Binary32: each workgroup takes a 2 * 256-element slice of pairs at a time.
__global__ __launch_bounds__(256) void fill_uniform_f32_kernel(float* out, int64_t count, uint64_t seed,
                                                               uint64_t counter0)
{
    const int64_t slice = 2 * 256 * 64;  // elements per workgroup slice (64 pairs per thread)
    for (int64_t s0 = (int64_t)blockIdx.x * slice; s0 < count; s0 += (int64_t)gridDim.x * slice) {
        const int64_t len = min(slice, count - s0);
        f32_stream<256>(seed, counter0 + (uint64_t)s0, len, threadIdx.x,
                        [&](int64_t j, float v) { out[s0 + j] = v; });
    }
}

sb_status run_fill_uniform(sb_handle* h, sb_dtype dt, void* out, int64_t count, uint64_t seed, uint64_t counter0)
{
    if (count == 0) return SB_OK;
    const int64_t blocks = std::min<int64_t>(4096, (count + 255) / 256);
    if (dt == SB_F64)
        hipLaunchKernelGGL(fill_uniform_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, h->stream,
                           static_cast<double*>(out), count, seed, counter0);
    else
        hipLaunchKernelGGL(fill_uniform_f32_kernel, dim3((unsigned)std::min<int64_t>(4096, (count + 32767) / 32768)),
                           dim3(256), 0, h->stream, static_cast<float*>(out), count, seed, counter0);
    return check_launch(h, dt == SB_F64 ? "fill_uniform_f64_kernel" : "fill_uniform_f32_kernel");
}

// ---- batched materialisation of GEMV requests -----------------------------
//
// One launch makes the operands of many requests: every block of rpi rows
// of every A is a work item (binary32 rows are generated in place; bfloat16
// rows are generated, reduced to their amax and encoded, exactly as
// sb_fill_uniform followed by sb_quantize_rows would produce them), plus one
// item per request for x (counters m*n ... m*n + n - 1) and the zeroed c.
// rpi is 1 for rows of SB_GEN_ITEM_ELEMS values or more and grows as rows
// get shorter, so that no item is much smaller than that many values: the
// cost of starting an item (finding its request, a chain of dependent
// loads) is then spread over a useful amount of work.
#ifndef SB_GEN_ITEM_ELEMS
#define SB_GEN_ITEM_ELEMS 4096
#endif

struct GenHeader {
    int64_t count, nitems, pad[6];
};
struct GenRec {
    int32_t dtype, rpi;  // rpi: rows per work item
    int64_t m, n, lda;
    uint64_t seed;
    void* A;
    float* scales;
    float* x;
    float* c;
    int64_t item0;
};
static_assert(sizeof(GenHeader) == 64 && sizeof(GenRec) == 80, "generator table layout");

// One wave per work item (four items per workgroup): items are small (the
// serving trace's median row is a few hundred values), so an item's
// overhead — finding its request and, for bfloat16, reducing each row's
// amax — stays inside the wave, with no workgroup barriers.  A bfloat16 row of up to
// kStashW values keeps its values in the wave's share of LDS between the
// amax pass and the encoding pass; longer rows are generated twice.  The
// row scale is a power of two, so dividing by it equals multiplying by its
// exact reciprocal whenever that reciprocal is a normal binary32 number.
#ifndef SB_GEN_STASH
#define SB_GEN_STASH 2048
#endif
constexpr int64_t kStashW = SB_GEN_STASH;  // 8 KiB per wave, 32 KiB per workgroup

// One bfloat16 row: generate it, reduce its amax, encode it with the row
// scale (rows of up to kStashW values are generated once, their values kept
// in the wave's LDS stash between the two passes).
__device__ __forceinline__ void bf16_row(const GenRec& r, int64_t row, uint64_t c0, float* st, int lane)
{
    const bool kept = r.n <= kStashW;
    float amax = 0.0f;
    f32_stream<kWave>(r.seed, c0, r.n, lane, [&](int64_t j, float v) {
        if (kept) st[j] = v;
        const float a = fabsf(v);
        if (a == a && a > amax) amax = a;
    });
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, kWave));
    const float s = row_scale(true, amax);
    const float inv = s >= 0x1.0p-126f ? 1.0f / s : 0.0f;
    if (lane == 0) r.scales[row] = s;
    uint16_t* Qr = static_cast<uint16_t*>(r.A) + row * r.lda;
    auto enc = [&](int64_t j, float v) { Qr[j] = bf16_encode(inv != 0.0f ? v * inv : v / s); };
    if (kept) {
        // the elements this lane stashed in the first pass
        const int64_t n = r.n;
        for_pairs<kWave>(c0, n, lane, [&](uint64_t, int64_t j) {
            if (j >= 0) enc(j, st[j]);
            if (j + 1 < n) enc(j + 1, st[j + 1]);
        });
    } else {
        f32_stream<kWave>(r.seed, c0, r.n, lane, enc);
    }
}

__global__ __launch_bounds__(256) void generate_kernel(const unsigned char* table)
{
    __shared__ float stash[256 / kWave][kStashW];
    const GenHeader* hdr = reinterpret_cast<const GenHeader*>(table);
    const GenRec* recs = reinterpret_cast<const GenRec*>(table + sizeof(GenHeader));
    const int64_t count = hdr->count, nitems = hdr->nitems;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (256 / kWave);
    for (int64_t item = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave; item < nitems; item += waves) {
        int64_t lo = 0, hi = count - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (recs[mid].item0 <= item) lo = mid;
            else hi = mid - 1;
        }
        const GenRec r = recs[lo];
        const int64_t blk = item - r.item0;
        // bfloat16 rows exist even when n = 0: their scale is 1, as the
        // quantiser gives a row whose largest magnitude is 0
        const int64_t rows = (r.n > 0 || r.dtype == SB_BF16) ? r.m : 0;
        if (blk * r.rpi < rows) {
            const int64_t r0 = blk * r.rpi, r1 = min(rows, r0 + r.rpi);
            if (r.dtype == SB_F32 && r.lda == r.n) {
                // consecutive rows are consecutive counters and addresses
                float* Ab = static_cast<float*>(r.A) + r0 * r.n;
                f32_stream<kWave>(r.seed, (uint64_t)(r0 * r.n), (r1 - r0) * r.n, lane,
                                  [&](int64_t j, float v) { Ab[j] = v; });
            } else {
                for (int64_t row = r0; row < r1; ++row) {
                    const uint64_t c0 = (uint64_t)(row * r.n);
                    if (r.dtype == SB_F32) {
                        float* Ar = static_cast<float*>(r.A) + row * r.lda;
                        f32_stream<kWave>(r.seed, c0, r.n, lane, [&](int64_t j, float v) { Ar[j] = v; });
                    } else {
                        bf16_row(r, row, c0, stash[threadIdx.x / kWave], lane);
                    }
                }
            }
        } else {
            const uint64_t c0 = (uint64_t)(r.m * r.n);
            f32_stream<kWave>(r.seed, c0, r.n, lane, [&](int64_t j, float v) { r.x[j] = v; });
            for (int64_t i = lane; i < r.m; i += kWave) r.c[i] = 0.0f;
        }
    }
}

}  // namespace sb

using sb::fail;

extern "C" {

size_t sb_generate_batched_bytes(int32_t count)
{
    return count < 0 ? (size_t)-1 : sizeof(sb::GenHeader) + (size_t)count * sizeof(sb::GenRec);
}

sb_status sb_generate_batched(sb_handle* handle, const sb_gen_desc* descs, int32_t count)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_generate_batched: NULL handle");
    if (count < 0 || (count > 0 && !descs)) return fail(handle, SB_EINVAL, "sb_generate_batched: bad descriptors");
    try {
        std::vector<unsigned char> image(sb_generate_batched_bytes(count));
        memset(image.data(), 0, image.size());
        auto* hdr = reinterpret_cast<sb::GenHeader*>(image.data());
        auto* recs = reinterpret_cast<sb::GenRec*>(image.data() + sizeof(sb::GenHeader));
        int64_t items = 0;
        for (int32_t k = 0; k < count; ++k) {
            const sb_gen_desc& d = descs[k];
            if ((d.dtype != SB_F32 && d.dtype != SB_BF16) || d.m < 0 || d.n < 0 || d.lda < (d.n > 1 ? d.n : 1) ||
                d.m > ((int64_t)1 << 31) || d.n > ((int64_t)1 << 31))
                return fail(handle, SB_EINVAL, "sb_generate_batched: descriptor %d: bad dtype, size or lda", k);
            const int es = d.dtype == SB_F32 ? 4 : 2;
            if ((d.m > 0 && d.n > 0 && !d.A) || (d.m > 0 && d.dtype == SB_BF16 && !d.scales) || (d.n > 0 && !d.x) ||
                (d.m > 0 && !d.c) || (uintptr_t)d.A % es || (uintptr_t)d.x % 4 || (uintptr_t)d.c % 4 ||
                (uintptr_t)d.scales % 4)
                return fail(handle, SB_EINVAL, "sb_generate_batched: descriptor %d: NULL or misaligned pointer", k);
            sb::GenRec& r = recs[k];
            r.dtype = d.dtype;
            r.m = d.m;
            r.n = d.n;
            r.lda = d.lda;
            r.seed = d.seed;
            r.A = d.A;
            r.scales = d.scales;
            r.x = d.x;
            r.c = d.c;
            r.item0 = items;
            const int64_t rows = (d.n > 0 || d.dtype == SB_BF16) ? d.m : 0;
            r.rpi = (int32_t)std::max<int64_t>(1, std::min<int64_t>(SB_GEN_ITEM_ELEMS / std::max<int64_t>(d.n, 1),
                                                                     std::max<int64_t>(rows, 1)));
            items += (rows + r.rpi - 1) / r.rpi + 1;  // the row blocks of A, then x and c
            (void)es;
        }
        hdr->count = count;
        hdr->nitems = items;
        if (items == 0) return SB_OK;
        if (image.size() > handle->ws_bytes || !sb::aligned16(handle->ws))
            return fail(handle, SB_ENOMEM, "sb_generate_batched needs %zu workspace bytes, handle has %zu",
                        image.size(), handle->ws_bytes);
        const hipError_t e = hipMemcpyAsync(sb::claim_ws(handle), image.data(), image.size(), hipMemcpyHostToDevice, handle->stream);
        if (e != hipSuccess) return fail(handle, SB_EDEVICE, "sb_generate_batched: copy: %s", hipGetErrorString(e));
        const int64_t grid = std::min<int64_t>((items + 3) / 4, 4096);  // four items (waves) per workgroup
        hipLaunchKernelGGL(sb::generate_kernel, dim3((unsigned)grid), dim3(256), 0, handle->stream,
                           static_cast<const unsigned char*>(handle->ws));
        return sb::check_launch(handle, "generate_kernel");
    } catch (...) {
        return fail(handle, SB_EINTERNAL, "sb_generate_batched: unexpected C++ exception");
    }
}

}  // extern "C"
