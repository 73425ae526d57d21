// On-device operand generation for the serving loop: counter-based uniform
// values in [-1, 1) from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).
// Element k of a fill is generated from counter c = counter0 + k:
//   z = seed + (c + 1) * 0x9E3779B97F4A7C15
//   z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
//   z = (z ^ (z >> 27)) * 0x94D049BB133111EB
//   z =  z ^ (z >> 31)
//   u = (z >> 11) * 2^-53 in [0, 1);  value = 2u - 1 (binary64, exact)
// binary32 outputs are the binary64 value rounded to nearest.  Generating
// operands where they are used keeps host-to-device copies off the request
// path; any element can be regenerated on its own from (seed, counter).
#include <algorithm>

#include "sb_device.hpp"
#include "sb_internal.hpp"

namespace sb {

__device__ __forceinline__ double splitmix_uniform(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    const double u = (double)(z >> 11) * 0x1.0p-53;
    return 2.0 * u - 1.0;
}

template <typename T>
__global__ __launch_bounds__(256) void fill_uniform_kernel(T* out, int64_t count, uint64_t seed, uint64_t counter0)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < count; k += stride)
        out[k] = (T)splitmix_uniform(seed, counter0 + (uint64_t)k);
}

sb_status run_fill_uniform(sb_handle* h, sb_dtype dt, void* out, int64_t count, uint64_t seed, uint64_t counter0)
{
    if (count == 0) return SB_OK;
    const int64_t blocks = std::min<int64_t>(4096, (count + 255) / 256);
    if (dt == SB_F64)
        hipLaunchKernelGGL(fill_uniform_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, h->stream,
                           static_cast<double*>(out), count, seed, counter0);
    else
        hipLaunchKernelGGL(fill_uniform_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, h->stream,
                           static_cast<float*>(out), count, seed, counter0);
    return check_launch(h, "fill_uniform_kernel");
}

}  // namespace sb
