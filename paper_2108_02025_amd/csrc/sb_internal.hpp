// Host-side internals of the streamblas library: the handle, error
// reporting, and the launch plans of each kernel family.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "streamblas.h"

struct sb_handle {
    void* ws;
    size_t ws_bytes;
    uint64_t ws_gen;  // advanced whenever a call writes the workspace (plans check it)
    hipStream_t stream;
    int64_t dot_small_bytes;      // SB_CUTOFF_DOT_SMALL_BYTES
    int64_t gemv_t_small_splits;  // SB_CUTOFF_GEMV_T_SMALL_SPLITS
    char err[512];
};

namespace sb {

// The workspace for a call that writes it: advances the handle's workspace
// generation, which invalidates a batched plan whose table lives there.
inline void* claim_ws(sb_handle* h)
{
    ++h->ws_gen;
    return h->ws;
}

// Record a formatted failure reason on the handle (or the thread-local
// slot when h is NULL) and return `st`.
sb_status fail(sb_handle* h, sb_status st, const char* fmt, ...)
    __attribute__((format(printf, 3, 4)));

// Check the result of a HIP launch or call.
sb_status check_launch(sb_handle* h, const char* what);

// ---- GEMV on a row-major view -------------------------------------------
// Every GEMV reduces to one of two kernels on a row-major rows x cols
// matrix with leading dimension ld:
//   "row-dot"   (kernel N): out[i] += sum_j M[i, j] v[j]     (out has rows entries)
//   "col-axpy"  (kernel T): out[j] += sum_i M[i, j] v[i]     (out has cols entries)
struct GemvNPlan {
    int G;          // lanes cooperating on one row (power of two, 4..64)
    int NT;         // threads per workgroup
    int64_t KC;     // columns per split (x chunk staged in LDS), multiple of 4
    int64_t nsplit; // number of column splits (1: no second stage)
    int64_t RB;     // rows per workgroup
    size_t lds;     // dynamic LDS bytes
    size_t ws;      // workspace bytes (split partial sums)
    int xcopies;    // copies of x in LDS: 1, or 16/esize shifted ones for rows not 16-byte aligned
    bool pairs;     // binary32 rows not aligned: two copies read as 8-byte pairs (xcopies 2)
};
GemvNPlan plan_gemv_n(int esize, int64_t rows, int64_t cols, bool unaligned = false);

struct GemvTPlan {
    int NT;         // threads per workgroup (waves split the rows of a split): 256, or
                    // 1024 for a small matrix done without a row split in one launch
    int64_t nsplit; // number of row splits
    int64_t RS;     // rows per split
    size_t ws;
};
GemvTPlan plan_gemv_t(int esize, int64_t rows, int64_t cols, int64_t small_splits);
extern const int64_t kDefaultGemvTSmallSplits;

sb_status run_gemv_n(sb_handle* h, sb_dtype dt, int64_t rows, int64_t cols, const void* M,
                     int64_t ld, const void* v, void* out);
sb_status run_gemv_t(sb_handle* h, sb_dtype dt, int64_t rows, int64_t cols, const void* M,
                     int64_t ld, const void* v, void* out);

// ---- two-sided GEMV -------------------------------------------------------
// out_r[i] += sum_j M[i, j] vc[j] and out_c[j] += sum_i M[i, j] vr[i] in one
// pass over a row-major rows x cols view M.
struct Gemv2Plan {
    int NW;             // waves per workgroup (each 64 lanes x 16 bytes of columns)
    int64_t ncb;        // column bands (partial row sums when > 1)
    int64_t nsplit;     // row bands (partial column sums when > 1)
    int64_t RS;         // rows per band
    size_t lds;         // dynamic LDS bytes
    size_t ws_c_offset; // workspace offset of the partial column sums
    size_t ws;          // workspace bytes
};
Gemv2Plan plan_gemv2(int esize, int64_t rows, int64_t cols);
sb_status run_gemv2(sb_handle* h, sb_dtype dt, int64_t rows, int64_t cols, const void* M, int64_t ld,
                    const void* vc, const void* vr, void* out_r, void* out_c);

// ---- DOT ------------------------------------------------------------------
struct DotPlan {
    bool small;     // one workgroup, one launch, no workspace
    int NT;
    int64_t nblocks;
    int64_t chunk;  // elements per workgroup, multiple of NT*4
    size_t ws;
};
DotPlan plan_dot(int esize, int64_t n, int partial_values, int64_t small_bytes);
extern const int64_t kDefaultDotSmallBytes;
sb_status run_dot(sb_handle* h, sb_dtype dt, int64_t n, const void* x, const void* y, void* alpha);
sb_status run_dot2(sb_handle* h, int64_t n, const float* x, const float* y, float* alpha);

// ---- GER ------------------------------------------------------------------
sb_status run_ger(sb_handle* h, sb_dtype dt, int64_t rows, int64_t cols, const void* x,
                  const void* y, void* C, int64_t ld);

// ---- precision form -------------------------------------------------------
sb_status run_quantize_rows(sb_handle* h, sb_dtype q, int64_t m, int64_t n, const float* A,
                            int64_t lda, void* Aq, int64_t ldq, float* scales);
sb_status run_gemv_q(sb_handle* h, sb_dtype q, int64_t m, int64_t n, const void* Aq, int64_t ldq,
                     const float* scales, const float* x, float* c);
size_t gemv_q_ws_bytes(sb_dtype q, int64_t m, int64_t n);
sb_status run_quantize_mx(sb_handle* h, sb_dtype q, int64_t m, int64_t n, const float* A, int64_t lda, void* Q,
                          int64_t ldq, uint8_t* S, int64_t lds);
sb_status run_gemv_mx(sb_handle* h, sb_dtype q, int64_t m, int64_t n, const void* Q, int64_t ldq, const uint8_t* S,
                      int64_t lds, const float* x, float* c);
size_t gemv_mx_ws_bytes(sb_dtype q, int64_t m, int64_t n);

// ---- operand generation ---------------------------------------------------
sb_status run_fill_uniform(sb_handle* h, sb_dtype dt, void* out, int64_t count, uint64_t seed, uint64_t counter0);

// ---- measurement probes ---------------------------------------------------
size_t probe_ws_bytes(size_t bytes);
sb_status run_stream_read(sb_handle* h, const void* src, size_t bytes);
sb_status run_stream_copy(sb_handle* h, const void* src, void* dst, size_t bytes);
sb_status run_stream_update(sb_handle* h, void* C, int64_t rows, int64_t cols, int64_t ld);

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace sb
