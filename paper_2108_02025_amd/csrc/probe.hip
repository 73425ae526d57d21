// Measurement probes: a streaming read and a streaming copy of a byte range
// with the same 16-byte non-temporal accesses and unrolling as the operation
// kernels.  They measure the practical HBM ceiling that the operations are
// compared against, and give a copy of known size for calibrating hardware
// traffic counters.
#include <algorithm>

#include "sb_device.hpp"
#include "sb_internal.hpp"

namespace sb {

#ifndef SB_PROBE_UNROLL
#define SB_PROBE_UNROLL 32
#endif
constexpr int kProbeNT = 256, kProbeUnroll = SB_PROBE_UNROLL;

// Each workgroup reads a contiguous chunk and folds it with XOR into one
// 16-byte value per workgroup (so the loads cannot be removed).
__global__ __launch_bounds__(kProbeNT) void stream_read_kernel(const v4u* src, int64_t n16,
                                                               int64_t chunk, v4u* sink)
{
    __shared__ v4u red[kProbeNT / kWave];
    const int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = min(n16, b0 + chunk);
    v4u acc = (v4u)0u;
    int64_t v = b0 + threadIdx.x;
    for (; v + (kProbeUnroll - 1) * kProbeNT < b1; v += kProbeUnroll * kProbeNT) {
        v4u t[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) t[u] = ld_stream(src + v + u * kProbeNT);
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) acc ^= t[u];
    }
    for (; v < b1; v += kProbeNT) acc ^= ld_stream(src + v);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        v4u o;
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = __shfl_xor(acc[q], off, kWave);
        acc ^= o;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        v4u t = red[0];
#pragma unroll
        for (int k = 1; k < kProbeNT / kWave; ++k) t ^= red[k];
        sink[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kProbeNT) void stream_copy_kernel(const v4u* src, v4u* dst, int64_t n16,
                                                               int64_t chunk)
{
    const int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = min(n16, b0 + chunk);
    int64_t v = b0 + threadIdx.x;
    for (; v + (kProbeUnroll - 1) * kProbeNT < b1; v += kProbeUnroll * kProbeNT) {
        v4u t[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) t[u] = ld_stream(src + v + u * kProbeNT);
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) st_stream(dst + v + u * kProbeNT, t[u]);
    }
    for (; v < b1; v += kProbeNT) st_stream(dst + v, ld_stream(src + v));
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

static void probe_geometry(int64_t n16, int64_t* blocks, int64_t* chunk)
{
    const int64_t step = (int64_t)kProbeNT * kProbeUnroll;
    int64_t g = std::max<int64_t>(1, std::min<int64_t>(2048, ceil_div(n16, step)));
    *chunk = ceil_div(ceil_div(n16, g), kProbeNT) * kProbeNT;
    *blocks = ceil_div(n16, *chunk);
}

size_t probe_ws_bytes(size_t bytes)
{
    int64_t blocks, chunk;
    if (bytes == 0) return 0;
    probe_geometry((int64_t)(bytes / 16), &blocks, &chunk);
    return (size_t)blocks * 16;
}

sb_status run_stream_read(sb_handle* h, const void* src, size_t bytes)
{
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return SB_OK;
    int64_t blocks, chunk;
    probe_geometry(n16, &blocks, &chunk);
    if ((size_t)blocks * 16 > h->ws_bytes)
        return fail(h, SB_ENOMEM, "stream_read needs %zu workspace bytes, handle has %zu", (size_t)blocks * 16,
                    h->ws_bytes);
    hipLaunchKernelGGL(stream_read_kernel, dim3((unsigned)blocks), dim3(kProbeNT), 0, h->stream,
                       static_cast<const v4u*>(src), n16, chunk, static_cast<v4u*>(claim_ws(h)));
    return check_launch(h, "stream_read_kernel");
}

sb_status run_stream_copy(sb_handle* h, const void* src, void* dst, size_t bytes)
{
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return SB_OK;
    int64_t blocks, chunk;
    probe_geometry(n16, &blocks, &chunk);
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(kProbeNT), 0, h->stream,
                       static_cast<const v4u*>(src), static_cast<v4u*>(dst), n16, chunk);
    return check_launch(h, "stream_copy_kernel");
}

}  // namespace sb
