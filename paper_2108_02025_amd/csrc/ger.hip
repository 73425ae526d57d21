// GER kernel: C += x (outer) y on a row-major view of C.
//
// Section 3.1 defines each entry as the elementary product x_i y_j added to
// the initial C_ij; section 4.2 (Algorithm 2) updates C row by row and notes
// that threading the inner loop would race on C.  Here every entry has
// exactly one owning lane: a lane owns W consecutive columns (y held in
// registers) and walks a block of rows, x_i being wave-uniform.  C streams
// in and out with 16-byte non-temporal loads and stores, several rows in
// flight per lane.  The product is rounded before the addition (no fused
// multiply-add), exactly as the definition states, so every entry is
// C_ij + fl(x_i y_j) regardless of the launch configuration.
#include <algorithm>

#include "sb_device.hpp"
#include "sb_internal.hpp"

namespace sb {

// Build-time launch constants (overridable with -D for tuning sweeps).
#ifndef SB_GER_UNROLL
#define SB_GER_UNROLL 32
#endif
#ifndef SB_GER_LOAD_NT
#define SB_GER_LOAD_NT 1
#endif
#ifndef SB_GER_STORE_NT
#define SB_GER_STORE_NT 1
#endif
#ifndef SB_GER_BLOCKS
#define SB_GER_BLOCKS 32768
#endif
#ifndef SB_GER_MIN_ROWS
#define SB_GER_MIN_ROWS 32
#endif
#ifndef SB_GER_COLS
#define SB_GER_COLS 1
#endif
constexpr int kUnrollGer = SB_GER_UNROLL;
constexpr int kGerCols = SB_GER_COLS;
constexpr bool kGerLoadNT = SB_GER_LOAD_NT, kGerStoreNT = SB_GER_STORE_NT;

template <typename T>
struct GerArgs {
    int64_t rows, cols, ld;
    const T* x;
    const T* y;
    T* C;
    int64_t RB;
    uint64_t mask;  // the update probe's XOR mask (0 at run time)
};

// The update probe's stand-in for the GER arithmetic: XOR of the bits with a
// mask that is 0 at run time (so C is rewritten unchanged, and the compiler
// cannot drop the load or the store).
template <typename V>
__device__ __forceinline__ V xor_bits(V v, uint64_t mask)
{
    typedef uint64_t u2 __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(V) == 16) {
        u2 b = __builtin_bit_cast(u2, v);
        b ^= mask;
        return __builtin_bit_cast(V, b);
    } else if constexpr (sizeof(V) == 8) {
        return __builtin_bit_cast(V, __builtin_bit_cast(uint64_t, v) ^ mask);
    } else {
        return __builtin_bit_cast(V, __builtin_bit_cast(uint32_t, v) ^ (uint32_t)mask);
    }
}

// PROBE: the measurement probe with GER's access pattern and launch shape
// (C read and rewritten in place, no arithmetic): the ceiling of the read +
// write stream GER moves.
template <typename T, int NT, bool ALIGNED, bool PROBE = false>
__global__ __launch_bounds__(NT) void ger_kernel(GerArgs<T> a)
{
    constexpr int W = ALIGNED ? Vec<T>::W : 1;
    typedef typename std::conditional<ALIGNED, typename Vec<T>::type, T>::type V;
    constexpr int U = kUnrollGer;
    constexpr int CH = ALIGNED ? kGerCols : 1;  // column chunks per lane, NT*W columns apart

    // This lane's chunks start at j0 + k * NT * W, k < CH.
    const int64_t j0 = (int64_t)blockIdx.x * NT * W * CH + (int64_t)threadIdx.x * W;
    if (j0 >= a.cols) return;
    const int64_t i0 = (int64_t)blockIdx.y * a.RB;
    const int64_t i1 = min(a.rows, i0 + a.RB);

    if (j0 + (int64_t)(CH - 1) * NT * W + W <= a.cols) {
        T yv[CH][W];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
#pragma unroll
            for (int q = 0; q < W; ++q) yv[k][q] = PROBE ? T(0) : a.y[j0 + (int64_t)k * NT * W + q];
        }
        int64_t i = i0;
        for (; i + U - 1 < i1; i += U) {
            V cv[U][CH];
            T xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int k = 0; k < CH; ++k)
                    cv[u][k] = ld_stream<kGerLoadNT>(
                        reinterpret_cast<const V*>(a.C + (i + u) * a.ld + j0 + (int64_t)k * NT * W));
                xv[u] = PROBE ? T(0) : a.x[i + u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    if constexpr (PROBE) {
                        cv[u][k] = xor_bits(cv[u][k], a.mask);
                    } else if constexpr (W == 1) {
                        cv[u][k] = add_rn(cv[u][k], mul_rn(xv[u], yv[k][0]));
                    } else {
#pragma unroll
                        for (int q = 0; q < W; ++q) cv[u][k][q] = add_rn(cv[u][k][q], mul_rn(xv[u], yv[k][q]));
                    }
                    st_stream<kGerStoreNT>(reinterpret_cast<V*>(a.C + (i + u) * a.ld + j0 + (int64_t)k * NT * W),
                                           cv[u][k]);
                }
            }
        }
        for (; i < i1; ++i) {
            const T xi = PROBE ? T(0) : a.x[i];
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                V* p = reinterpret_cast<V*>(a.C + i * a.ld + j0 + (int64_t)k * NT * W);
                V cv = ld_stream<kGerLoadNT>(p);
                if constexpr (PROBE) {
                    cv = xor_bits(cv, a.mask);
                } else if constexpr (W == 1) {
                    cv = add_rn(cv, mul_rn(xi, yv[k][0]));
                } else {
#pragma unroll
                    for (int q = 0; q < W; ++q) cv[q] = add_rn(cv[q], mul_rn(xi, yv[k][q]));
                }
                st_stream<kGerStoreNT>(p, cv);
            }
        }
    } else {
        // Right edge: element by element over this lane's columns.
        for (int k = 0; k < CH; ++k) {
            const int64_t jk = j0 + (int64_t)k * NT * W;
            const int64_t rem = min<int64_t>(W, a.cols - jk);
            for (int64_t i = i0; i < i1; ++i) {
                const T xi = PROBE ? T(0) : a.x[i];
                for (int64_t q = 0; q < rem; ++q) {
                    T* p = a.C + i * a.ld + jk + q;
                    *p = PROBE ? xor_bits(*p, a.mask) : add_rn(*p, mul_rn(xi, a.y[jk + q]));
                }
            }
        }
    }
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename T, bool PROBE = false>
static sb_status ger_typed(sb_handle* h, int64_t rows, int64_t cols, const T* x, const T* y, T* C,
                           int64_t ld)
{
    constexpr int NT = 256;
    const bool al = aligned16(C) && ((ld * (int64_t)sizeof(T)) % 16 == 0);
    const int64_t W = al ? 16 / (int64_t)sizeof(T) : 1;
    const int64_t cblocks = ceil_div(cols, NT * W * (al ? kGerCols : 1));
    // Aim for about 128 workgroups per compute unit over the whole launch,
    // each streaming at least SB_GER_MIN_ROWS rows.
    const int64_t target = SB_GER_BLOCKS;
    int64_t rb = std::max<int64_t>(SB_GER_MIN_ROWS, ceil_div(rows, std::max<int64_t>(1, target / cblocks)));
    rb = std::min<int64_t>(rb, rows);
    GerArgs<T> a{rows, cols, ld, x, y, C, rb, 0};
    const dim3 grid((unsigned)cblocks, (unsigned)ceil_div(rows, rb));
    if (al) hipLaunchKernelGGL((ger_kernel<T, NT, true, PROBE>), grid, dim3(NT), 0, h->stream, a);
    else hipLaunchKernelGGL((ger_kernel<T, NT, false, PROBE>), grid, dim3(NT), 0, h->stream, a);
    return check_launch(h, PROBE ? "ger_kernel (update probe)" : "ger_kernel");
}

sb_status run_ger(sb_handle* h, sb_dtype dt, int64_t rows, int64_t cols, const void* x,
                  const void* y, void* C, int64_t ld)
{
    if (rows == 0 || cols == 0) return SB_OK;
    if (dt == SB_F64)
        return ger_typed<double>(h, rows, cols, static_cast<const double*>(x),
                                 static_cast<const double*>(y), static_cast<double*>(C), ld);
    return ger_typed<float>(h, rows, cols, static_cast<const float*>(x), static_cast<const float*>(y),
                            static_cast<float*>(C), ld);
}

sb_status run_stream_update(sb_handle* h, void* C, int64_t rows, int64_t cols, int64_t ld)
{
    if (rows == 0 || cols == 0) return SB_OK;
    return ger_typed<double, true>(h, rows, cols, nullptr, nullptr, static_cast<double*>(C), ld);
}

}  // namespace sb
