/*
 * streamblas: GEMV, DOT and GER for one AMD Instinct MI355X (gfx950).
 *
 * The operations and their names follow A. Singh and C. Bassoy, "High
 * Performance Level-1 and Level-2 BLAS" (arXiv 2108.02025):
 *   DOT   alpha += x . y        section 3.1, Definition (DOT); section 4.3
 *   GER   C += x (outer) y      section 3.1, Definition (GEM); section 4.2
 *   GEMV  c += A x, c += A^T x  section 3.1, Definition (GEMV); sections 4.1-4.2
 * Every operation accumulates into its output: the products are summed first
 * and the initial output value is added once, at the end.  There is no BLAS
 * alpha/beta scaling; alpha is DOT's accumulator.
 *
 * Memory and streams.  Every pointer argument named A, x, y, c, C, alpha,
 * Aq, scales or workspace is a DEVICE pointer owned by the caller.  The
 * library never allocates device memory; kernels that need scratch (split
 * reductions) use the workspace given to the handle.  Each call only
 * enqueues work on the handle's HIP stream and returns; results are valid
 * once that stream is synchronised.  Launch failures are reported as
 * SB_EDEVICE; faults during execution surface at the caller's next
 * synchronisation.  A handle must be used by one host thread at a time.
 *
 * Layouts.  A is m x n.  Row-major element (i, j) is A[i*lda + j] with
 * lda >= max(1, n); column-major is A[i + j*lda] with lda >= max(1, m).
 * Vectors are contiguous (unit stride).  Sizes are 64-bit.
 *
 * Errors.  Functions return SB_OK (0) or a negative status; they never throw.
 * Argument checks run before any device work, so an invalid call enqueues
 * nothing.  sb_last_error() gives a readable reason for the last failure on
 * a handle.
 */
#ifndef STREAMBLAS_H
#define STREAMBLAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sb_status;

#define SB_OK 0
#define SB_EINVAL (-1)        /* invalid argument: size, stride, null pointer, overlap */
#define SB_ENOMEM (-2)        /* the handle's workspace is smaller than the call needs */
#define SB_EDEVICE (-3)       /* the HIP runtime refused a launch or query */
#define SB_EUNSUPPORTED (-4)  /* valid arguments, combination not implemented */
#define SB_EINTERNAL (-5)     /* unexpected internal failure */

typedef enum { SB_F64 = 0, SB_F32 = 1, SB_BF16 = 2, SB_FP8_E4M3 = 3, SB_MXFP8_E4M3 = 4,
               SB_MXFP4_E2M1 = 5 } sb_dtype;
typedef enum { SB_ROW_MAJOR = 0, SB_COL_MAJOR = 1 } sb_layout;
typedef enum { SB_N = 0, SB_T = 1 } sb_op;

/* Operation kinds, for sb_workspace_bytes. */
typedef enum { SB_KIND_GEMV = 0, SB_KIND_DOT = 1, SB_KIND_GER = 2, SB_KIND_GEMV_Q = 3,
               SB_KIND_DOT2 = 4, SB_KIND_PROBE_READ = 5, SB_KIND_GEMV2 = 6, SB_KIND_GEMV_MX = 7 } sb_kind;

typedef struct sb_handle sb_handle;

/* Library version (major*10000 + minor*100 + patch). */
int32_t sb_version(void);

/* Static text for a status code; never NULL. */
const char* sb_status_string(sb_status status);

/*
 * Create a handle.  workspace: device buffer of ws_bytes bytes (may be NULL
 * with ws_bytes = 0; calls that need scratch then fail with SB_ENOMEM).
 * stream: a hipStream_t, or NULL for the default stream.  The handle keeps
 * both pointers; the caller keeps ownership and must keep them alive while
 * the handle uses them.  No HIP call is made here.  *out receives the handle.
 */
sb_status sb_handle_create(void* workspace, size_t ws_bytes, void* stream, sb_handle** out);

/* Destroy a handle (NULL is accepted).  Does not free the workspace. */
sb_status sb_handle_destroy(sb_handle* handle);

/* Replace the stream used by later calls on this handle. */
sb_status sb_set_stream(sb_handle* handle, void* stream);

/* Replace the workspace used by later calls.  Work already enqueued may
 * still use the old buffer until the stream reaches it. */
sb_status sb_set_workspace(sb_handle* handle, void* workspace, size_t ws_bytes);

/* Text describing the last failure on this handle ("" if none); with a
 * NULL handle, the last failure of sb_handle_create on this thread. */
const char* sb_last_error(const sb_handle* handle);

/*
 * Small-problem cutoffs (section 4.3: below a size found by experiment, the
 * dot product runs without a parallel split; section 4 also advises fewer
 * parallel parts for small problems).  Each handle starts with the defaults
 * measured on MI355X; callers may re-measure and override them.
 *   SB_CUTOFF_DOT_SMALL_BYTES     sb_dot and sb_dot2_f32 with at most this
 *                                 many operand bytes (x and y together) run
 *                                 as one workgroup in a single launch that
 *                                 also adds alpha, with no workspace;
 *                                 above it, the two-stage form.
 *   SB_CUTOFF_GEMV_T_SMALL_SPLITS a column-axpy GEMV (row-major T,
 *                                 column-major N) whose row split would have
 *                                 2 .. this many parts runs unsplit with 16
 *                                 waves per column block in a single launch.
 * value must be >= 0 (0 disables the small path); SB_EINVAL otherwise.  A
 * cutoff changes the summation order (still deterministic for a given
 * shape and handle) and the workspace a call needs.
 */
typedef enum { SB_CUTOFF_DOT_SMALL_BYTES = 0, SB_CUTOFF_GEMV_T_SMALL_SPLITS = 1 } sb_cutoff;
sb_status sb_set_cutoff(sb_handle* handle, sb_cutoff which, int64_t value);
/* *value receives the handle's cutoff, or the default when handle is NULL. */
sb_status sb_get_cutoff(const sb_handle* handle, sb_cutoff which, int64_t* value);

/*
 * Workspace bytes that one call of the given kind and shape needs with this
 * handle's current tuning (0 if none).  For SB_KIND_DOT and SB_KIND_DOT2 the
 * length is n (m is ignored); for SB_KIND_GER the result is always 0; for
 * SB_KIND_GEMV2 op is ignored.
 * Returns (size_t)-1 for invalid arguments.
 */
size_t sb_workspace_bytes(const sb_handle* handle, sb_kind kind, sb_dtype dtype,
                          sb_layout layout, sb_op op, int64_t m, int64_t n);

/*
 * GEMV: c += op(A) x   (section 3.1, Definition (GEMV); section 4.1
 * Algorithm 1 for the column-major form, section 4.2 Algorithm 2 for the
 * row-major form).
 *   dtype  SB_F64 or SB_F32: A, x and c all have this type; products and
 *          sums are computed in it (fused multiply-add).  SB_BF16 and
 *          SB_FP8_E4M3 return SB_EUNSUPPORTED (use sb_gemv_q).
 *   op     SB_N: x has n entries, c has m.  SB_T: x has m entries, c has n.
 * (row-major, N) and (column-major, T) on the same buffer are the same
 * computation and give identical bits; so do (row-major, T) and
 * (column-major, N).  If the output length is 0 nothing is launched; if the
 * reduction length is 0, c is unchanged.  c must not overlap A or x.
 * Results are deterministic: the summation order depends only on
 * (dtype, layout, op, m, n, lda alignment) and the handle's tuning.
 */
sb_status sb_gemv(sb_handle* handle, sb_dtype dtype, sb_layout layout, sb_op op,
                  int64_t m, int64_t n, const void* A, int64_t lda,
                  const void* x, void* c);

/*
 * GEMV that allocates nothing, for callers that cannot allocate device
 * memory or lend the library a workspace: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * checks, kernels and result bits as sb_gemv on the same handle, but the
 * split partial sums go to a static device array of SB_NOALLOC_SCRATCH_BYTES
 * inside the library instead of the handle's workspace, which is neither
 * needed nor touched (batched plans on the handle stay valid).
 *   - One array per GPU: that of the device of the handle's stream.  Its
 *     device address is looked up (no allocation) on the first call that
 *     needs it on that device; the array lives until the process ends.
 *   - Every call on a GPU shares that GPU's array.  Calls that may overlap
 *     on one GPU (on different streams, or from several host threads) race
 *     and give wrong results: serialise them.  Calls in order on one stream
 *     are safe; the array keeps the last call's partial sums and nothing in
 *     it needs clearing (every partial sum is written before it is read).
 *   - A shape whose partial sums need more than SB_NOALLOC_SCRATCH_BYTES
 *     (sb_workspace_bytes of kind SB_KIND_GEMV) returns SB_ENOMEM before any
 *     HIP call.  Every other error is as for sb_gemv.
 */
#define SB_NOALLOC_SCRATCH_BYTES ((size_t)4 << 20)
sb_status sb_gemv_noalloc(sb_handle* handle, sb_dtype dtype, sb_layout layout, sb_op op,
                          int64_t m, int64_t n, const void* A, int64_t lda,
                          const void* x, void* c);

/*
 * Two-sided GEMV: c += A x and d += A^T y in one pass over A.  An extension
 * of the section 3.1 GEMV definition for callers that need both products of
 * one matrix (as in bidiagonalisation, or the BLAS Technical Forum's fused
 * GEMVT): the paper finds these operations bound by memory traffic
 * (sections 4.2 and 4.3), and reading A once instead of twice halves it.
 *   dtype  SB_F64 or SB_F32 for A, x, y, c and d.
 *   A      m x n in `layout` with leading dimension lda (as in sb_gemv).
 *   x      n entries; c: m entries, c_i += sum_j A_ij x_j.
 *   y      m entries; d: n entries, d_j += sum_i A_ij y_i.
 * Each output is the sum of its products with the initial value added last,
 * each sum in a fixed order that depends only on (dtype, layout, m, n, lda
 * alignment): deterministic, but not the same order as sb_gemv, so the bits
 * may differ from two sb_gemv calls within the same error bound.  x and y
 * may alias each other; c and d must not overlap A, x, y or each other
 * (SB_EINVAL).  If m or n is 0 nothing is launched and both outputs are
 * unchanged (an empty sum adds nothing).  Needs sb_workspace_bytes of kind
 * SB_KIND_GEMV2 in the handle's workspace (SB_ENOMEM otherwise).
 */
sb_status sb_gemv2(sb_handle* handle, sb_dtype dtype, sb_layout layout, int64_t m, int64_t n,
                   const void* A, int64_t lda, const void* x, const void* y, void* c, void* d);

/*
 * DOT: *alpha += x . y   (section 3.1, Definition (DOT); section 4.3,
 * Algorithms 3 and 4).  dtype SB_F64 or SB_F32; x and y have n entries;
 * alpha points to ONE device scalar of that type.  The products are summed
 * in a fixed two-stage order (per-workgroup partial sums in the workspace,
 * then one workgroup combines them in index order) and the initial alpha is
 * added last; below SB_CUTOFF_DOT_SMALL_BYTES one workgroup does all of it
 * in a single launch (Algorithm 3's small-problem form).  n = 0 leaves
 * alpha unchanged.  Deterministic for a given n and cutoff.
 */
sb_status sb_dot(sb_handle* handle, sb_dtype dtype, int64_t n, const void* x,
                 const void* y, void* alpha);

/*
 * GER: C += x (outer) y   (section 3.1, Definition (GEM); section 4.2,
 * Algorithm 2).  C is m x n in the given layout with leading dimension ldc;
 * x has m entries, y has n.  Each entry is computed as C_ij + fl(x_i y_j)
 * (the product rounded, then the addition), exactly as the definition
 * states, so the result does not depend on the launch configuration.
 * dtype SB_F64 or SB_F32.  C must not overlap x or y.
 */
sb_status sb_ger(sb_handle* handle, sb_dtype dtype, sb_layout layout, int64_t m,
                 int64_t n, const void* x, const void* y, void* C, int64_t ldc);

/*
 * Per-row scaled quantisation (precision form; the paper leaves the element
 * width generic).  A: m x n binary32, row-major, leading dimension lda.
 * Output: codes Aq (row-major, leading dimension ldq, in elements) and
 * scales[m] (binary32).  q = SB_BF16: s_i = 2^floor(log2 amax_i) and
 * 2-byte bfloat16 codes; q = SB_FP8_E4M3: s_i = amax_i / 448 and 1-byte
 * OCP E4M3FN codes, saturated to +-448.  amax_i is the largest |a_ij| over
 * non-NaN entries; a row whose amax is 0 or infinite gets s_i = 1.  Each
 * code is the round-to-nearest-even encoding of fl32(a_ij / s_i).
 */
sb_status sb_quantize_rows(sb_handle* handle, sb_dtype q, int64_t m, int64_t n,
                           const float* A, int64_t lda, void* Aq, int64_t ldq,
                           float* scales);

/*
 * Quantised GEMV: c_i += s_i * sum_j q_ij x_j with q decoded from Aq
 * (row-major, leading dimension ldq elements), x and c binary32, products
 * and sums in binary32 (fused multiply-add), the scale applied once per row
 * after the reduction.  q = SB_BF16 or SB_FP8_E4M3.
 */
sb_status sb_gemv_q(sb_handle* handle, sb_dtype q, int64_t m, int64_t n, const void* Aq,
                    int64_t ldq, const float* scales, const float* x, float* c);

/*
 * Microscaled storage of A (OCP Microscaling Formats v1.0; the paper's
 * element size S_data is generic and its GEMV bound by the bytes of A,
 * sections 4.1 and 4.3).  Each row is cut into blocks of 32 consecutive
 * elements (the last one may be shorter); a block has one E8M0 scale byte,
 * X = 2^(code - 127) (code 255 is NaN), and element codes P_j:
 *   q = SB_MXFP8_E4M3: OCP E4M3 codes, one byte per element;
 *   q = SB_MXFP4_E2M1: OCP E2M1 codes (magnitudes 0, .5, 1, 1.5, 2, 3, 4, 6),
 *                      element 2k in the low nibble of byte k of the row, an
 *                      unused last high nibble 0.
 * Element j of row i decodes to X_i,j/32 * P_ij.
 * Layout: Q row-major with ldq bytes per row (ldq >= the row's code bytes
 * and a multiple of 16; Q 16-byte aligned); S row-major, lds >= ceil(n/32)
 * scale bytes per row.  Both are device memory owned by the caller.
 *
 * sb_quantize_mx: codes and scales of the binary32 m x n matrix A (lda):
 * per block, code = clamp(floor(log2 amax) - emax + 127, 0, 254) with emax
 * = 8 (E4M3) or 2 (E2M1), 0 for an all-zero block, 255 (and element codes
 * 0) for a block holding a NaN or infinity; P_j = a_j / X rounded to
 * nearest even and saturated to the largest finite element value.  A, Q and
 * S must not overlap.
 *
 * sb_gemv_mx: c += (X * P) x with x (n entries) and c (m entries) binary32,
 * products and sums in binary32 (each block's partial sum scaled by its X).
 * c must not overlap Q, S or x.  Needs sb_workspace_bytes of kind
 * SB_KIND_GEMV_MX (dtype q) when rows are longer than 32768 elements.
 * Both return SB_EINVAL for other q, strides below the minimum or a
 * misaligned Q, and SB_OK without launching when m or n is 0.
 */
sb_status sb_quantize_mx(sb_handle* handle, sb_dtype q, int64_t m, int64_t n, const float* A, int64_t lda,
                         void* Q, int64_t ldq, uint8_t* S, int64_t lds);
sb_status sb_gemv_mx(sb_handle* handle, sb_dtype q, int64_t m, int64_t n, const void* Q, int64_t ldq,
                     const uint8_t* S, int64_t lds, const float* x, float* c);

/*
 * Compensated DOT in binary32: *alpha += x . y evaluated with error-free
 * transformations (TwoProduct through fused multiply-add, TwoSum) at every
 * step and every level of the reduction, as in the Dot2 algorithm of Ogita,
 * Rump and Oishi (SIAM J. Sci. Comput. 26(6), 2005).  The result is about as
 * accurate as a binary32 evaluation carried out in twice the working
 * precision.  alpha is one device binary32 scalar.
 */
sb_status sb_dot2_f32(sb_handle* handle, int64_t n, const float* x, const float* y,
                      float* alpha);

/*
 * Batched GEMV (batching form).  The paper notes that for small problems the
 * cost of starting threads dominates (section 4.2); on the GPU that cost is
 * a launch, so many problems c += op(A) x share one persistent launch.
 * layout and op have sb_gemv's meaning (m x n matrix A, lda its leading
 * dimension; op SB_N: x has n entries and c m, SB_T: x m and c n).
 *
 * Row dots (row-major N, column-major T: the output runs along the stored
 * rows) are cut into tiles of rows_per_tile stored rows by one column chunk
 * (split chunks per row; split > 1 is split-K: per-chunk partial sums are
 * added in chunk order, then the initial c).  Column axpys (row-major T,
 * column-major N: the output runs along the stored columns; sections 4.1
 * and 4.2) are cut into column blocks of one wave's width (256 binary32 or
 * 128 binary64 columns, or 64 if the stored rows are not 16-byte aligned)
 * by chunks of rows_per_tile stored rows (split chunks; partial sums added
 * in chunk order, then the initial c).
 * Runs of consecutive tiles of one problem form work items, which the
 * encoder deals to the workgroups of a fixed grid, largest first in rounds
 * of alternating direction, so the workgroups' shares differ by at most one
 * item.  A problem's result depends only on the problem and its
 * configuration, so it is bit-identical alone and in any mix.  Row dots use
 * the same per-row arithmetic as sb_gemv / sb_gemv_q.
 *
 *   dtype  SB_F64 or SB_F32: A, x and c of that type.  SB_BF16 or
 *          SB_FP8_E4M3 (row-major N only, else SB_EUNSUPPORTED): A holds
 *          codes (lda in elements) with per-row binary32 scales as written
 *          by sb_quantize_rows; x and c are binary32 and
 *          c_i += s_i * sum_j q_ij x_j.
 *   group  row dots: lanes cooperating on a row, 4, 8, 16, 32 or 64 (0:
 *          automatic).  Column axpys: must be 0.
 *   rows_per_tile  row dots: a multiple of 4 * (64 / group) (0: automatic,
 *          about 256 KiB of A per tile and at most 8 row passes of a
 *          workgroup; the tile height never changes a row's result).
 *          Column axpys: stored rows per chunk (0: from split, or about
 *          256 KiB of A per tile); the chunking sets the summation order.
 *   split  row dots: column chunks, each chunk's x must fit 64 KiB of LDS
 *          (0: automatic; for SB_F32, SB_BF16 and SB_FP8_E4M3 rows that
 *          are not all 16-byte aligned, chunks of at most 8192 columns, and
 *          a smaller split is raised to that: x is staged as two shifted
 *          copies).
 *          Column axpys: row chunks (0: from rows_per_tile; if both are
 *          given they must agree).
 * Outputs of different problems must not overlap.  Problems with m = 0 or
 * n = 0 are skipped.  The zero-initialised layout and op are row-major N.
 */
typedef struct {
    int32_t dtype;
    int32_t group;
    int32_t rows_per_tile;
    int32_t split;
    int64_t m, n, lda;
    const void* A;
    const float* scales;
    const void* x;
    void* c;
    int32_t layout;  /* sb_layout */
    int32_t op;      /* sb_op */
} sb_gemv_desc;

/* Device bytes of the batch table (header, problem records, work items and
 * the per-workgroup item lists, second-stage items and split scratch) for these
 * descriptors; *image_bytes (if not NULL)
 * receives the size of the part sb_gemv_batched_encode writes.  Returns
 * (size_t)-1 for invalid descriptors. */
size_t sb_gemv_batched_table_bytes(const sb_gemv_desc* descs, int32_t count, size_t* image_bytes);

/* Copy the descriptors to out with every automatic field (0) replaced by
 * the value the batched kernel will use. */
sb_status sb_gemv_batched_resolve(const sb_gemv_desc* descs, int32_t count, sb_gemv_desc* out);

/* Write the table image for a table that will live at device address
 * dev_table (16-byte aligned, sb_gemv_batched_table_bytes bytes) into the
 * HOST buffer host_image (image_bytes long).  The caller copies the image to
 * dev_table before sb_gemv_batched_run.  No HIP call is made. */
sb_status sb_gemv_batched_encode(const sb_gemv_desc* descs, int32_t count, void* dev_table,
                                 void* host_image, size_t image_bytes);

/* Launch the persistent kernel over the table at dev_table on the handle's
 * stream (grid workgroups; 0 = 1024, the grid the items are dealt to; a
 * smaller grid runs several workgroups' lists per workgroup), then the
 * second-stage kernel that adds the split problems' partial sums in split
 * order (it returns at once if the table has none).  Everything the kernels
 * need is read from the table, so a captured launch can be replayed over new
 * tables written to the same address.  The table stays valid for further
 * launches. */
sb_status sb_gemv_batched_run(sb_handle* handle, const void* dev_table, int32_t grid);

/* Encode, copy the table into the handle's workspace (needs
 * sb_gemv_batched_table_bytes) and run, all on the handle's stream. */
sb_status sb_gemv_batched(sb_handle* handle, const sb_gemv_desc* descs, int32_t count);

/*
 * Batched plans: the descriptors are checked, resolved and encoded once; the
 * table is copied (on the handle's stream) into the handle's workspace,
 * which must hold sb_gemv_batched_table_bytes; sb_plan_run then launches the
 * persistent kernel on the handle's current stream with no host work, as
 * often as wanted (a captured sb_plan_run can be replayed).  The table
 * belongs to the plan: a later call on the same handle that writes the
 * workspace (a split GEMV, a two-stage DOT, another batch or plan, a probe,
 * the generator) or a new workspace makes sb_plan_run fail with SB_EINVAL
 * until the plan is created again.  Calls on the handle that need no
 * workspace leave the plan valid.  A plan must be destroyed before its
 * handle; sb_plan_destroy(NULL) is accepted.  A batch with no work gives a
 * plan whose runs launch nothing.
 */
typedef struct sb_plan sb_plan;
sb_status sb_plan_create(sb_handle* handle, const sb_gemv_desc* descs, int32_t count, sb_plan** out);
sb_status sb_plan_run(sb_plan* plan);
sb_status sb_plan_destroy(sb_plan* plan);

/*
 * Operand generation (serving form: requests' operands are made on the
 * device where they are used).  z = SplitMix64(seed, counter0 + k)
 * (Steele, Lea and Flood, OOPSLA 2014: z = seed + (c+1)*0x9E3779B97F4A7C15,
 * then the xor-shift-multiply finaliser with 0xBF58476D1CE4E5B9 and
 * 0x94D049BB133111EB).  dtype SB_F64: element e = counter0 + k is 2u - 1
 * with u = (z_e >> 11) * 2^-53.  SB_F32: two elements per state, element e
 * is (f - 2^23) * 2^-23 with f = z_(e>>1) >> 40 for even e and
 * (z_(e>>1) >> 8) & 0xFFFFFF for odd e (exact in binary32, no binary64
 * arithmetic).  Both lie in [-1, 1).  out must be aligned to the element
 * size; count >= 0; for SB_F32 the counters counter0 .. counter0 + count - 1
 * must not wrap past 2^64 (SB_EINVAL).
 */
sb_status sb_fill_uniform(sb_handle* handle, sb_dtype dtype, void* out, int64_t count, uint64_t seed,
                          uint64_t counter0);

/*
 * Batched operand generation for GEMV requests (serving form).  For each
 * descriptor: A (m x n row-major, lda elements) gets element (i, j) from
 * counter i*n + j, x gets element j from counter m*n + j (values as
 * sb_fill_uniform with the descriptor's seed), c is set to zero.  dtype
 * SB_F32 stores binary32 A; SB_BF16 stores the bfloat16 codes and per-row
 * scales that sb_quantize_rows would make from that binary32 A (bit for
 * bit; with n = 0 every scale is 1).  One launch on the handle's stream; the descriptors are copied into
 * the workspace first (sb_generate_batched_bytes bytes).  Work items are
 * blocks of rows of about 4096 values (a single row when rows are longer).
 */
typedef struct {
    int32_t dtype;
    int32_t reserved;
    int64_t m, n, lda;
    uint64_t seed;
    void* A;
    float* scales;
    float* x;
    float* c;
} sb_gen_desc;

size_t sb_generate_batched_bytes(int32_t count);
sb_status sb_generate_batched(sb_handle* handle, const sb_gen_desc* descs, int32_t count);

/*
 * Measurement probes (not operations of the paper).  They stream a byte
 * range with the same 16-byte non-temporal accesses as the operation
 * kernels, giving the practical HBM ceiling the operations are measured
 * against and a transfer of known size for calibrating hardware traffic
 * counters.  src and dst must be 16-byte aligned and bytes a multiple of
 * 16; the ranges must not overlap (SB_EINVAL otherwise).
 *   sb_stream_read: reads bytes from src; needs sb_workspace_bytes of kind
 *                   SB_KIND_PROBE_READ (m ignored, n = bytes) in the
 *                   workspace, where it leaves one XOR fold per workgroup.
 *   sb_stream_copy: copies bytes from src to dst; needs no workspace.
 */
sb_status sb_stream_read(sb_handle* handle, const void* src, size_t bytes);
sb_status sb_stream_copy(sb_handle* handle, const void* src, void* dst, size_t bytes);

/*
 * Read-and-rewrite probe with GER's access pattern: the rows x cols
 * row-major binary64 matrix C (leading dimension ldc >= cols, 8-byte
 * aligned) is read and written back unchanged, in place, by the GER kernel
 * with its arithmetic replaced by an XOR with a zero mask, in GER's launch
 * shape (section 4.2, Algorithm 2's row-by-row update).  It moves exactly the
 * bytes of C that GER moves, so its rate is the ceiling of GER's read +
 * write stream.  Needs no workspace.  SB_EINVAL for a NULL or misaligned C
 * or a bad size; nothing is launched for an empty matrix.
 */
sb_status sb_stream_update(sb_handle* handle, void* C, int64_t rows, int64_t cols, int64_t ldc);

#ifdef __cplusplus
}
#endif

#endif /* STREAMBLAS_H */
