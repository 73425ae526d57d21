// The C-ABI of streamblas: argument validation, the mapping of
// (layout, op) onto the two GEMV kernels, and error reporting.  Every check
// here runs before any HIP call, so a rejected call enqueues nothing.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>

#include "sb_internal.hpp"

namespace {

thread_local char g_err[512] = "";

const char* kStatusText[] = {
    "success",
    "invalid argument",
    "workspace too small",
    "HIP runtime error",
    "unsupported combination",
    "internal error",
};

bool mul_ok(int64_t a, int64_t b, int64_t* out) { return !__builtin_mul_overflow(a, b, out); }

int esize_of(sb_dtype dt)
{
    switch (dt) {
    case SB_F64: return 8;
    case SB_F32: return 4;
    case SB_BF16: return 2;
    case SB_FP8_E4M3: return 1;
    case SB_MXFP8_E4M3:
    case SB_MXFP4_E2M1: return 0;  // block-scaled codes: sizes come from mx_row_bytes
    }
    return 0;
}

// Number of elements spanned by a rows x cols matrix with leading dimension
// ld (row-major view), or -1 on overflow.  0 for an empty matrix.
int64_t span_elems(int64_t rows, int64_t cols, int64_t ld)
{
    if (rows == 0 || cols == 0) return 0;
    int64_t t;
    if (!mul_ok(rows - 1, ld, &t) || __builtin_add_overflow(t, cols, &t)) return -1;
    return t;
}

struct Range {
    uintptr_t lo, hi;  // [lo, hi) in bytes; empty when lo == hi
};

Range range_of(const void* p, int64_t elems, int es)
{
    const uintptr_t lo = reinterpret_cast<uintptr_t>(p);
    return Range{lo, lo + (uintptr_t)elems * (uintptr_t)es};
}

bool overlap(Range a, Range b) { return a.lo < a.hi && b.lo < b.hi && a.lo < b.hi && b.lo < a.hi; }

// Storage-only element types: GEMV, DOT and GER compute in binary64 or
// binary32; narrow codes go through the quantised and MX entry points.
bool narrow(sb_dtype dt)
{
    return dt == SB_BF16 || dt == SB_FP8_E4M3 || dt == SB_MXFP8_E4M3 || dt == SB_MXFP4_E2M1;
}

bool is_mx(sb_dtype q) { return q == SB_MXFP8_E4M3 || q == SB_MXFP4_E2M1; }

// Bytes of one row of MX element codes: n (E4M3) or ceil(n/2) (E2M1).
int64_t mx_row_bytes(sb_dtype q, int64_t n) { return q == SB_MXFP8_E4M3 ? n : (n + 1) / 2; }

bool misaligned(const void* p, int es) { return (reinterpret_cast<uintptr_t>(p) % (uintptr_t)es) != 0; }

constexpr int64_t kMaxBytes = (int64_t)1 << 46;  // 64 TiB: far above any device

}  // namespace

namespace sb {

sb_status fail(sb_handle* h, sb_status st, const char* fmt, ...)
{
    char* buf = h ? h->err : g_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
    return st;
}

sb_status check_launch(sb_handle* h, const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return SB_OK;
    return fail(h, SB_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace sb

using sb::fail;

#define SB_GUARD_BEGIN try {
#define SB_GUARD_END                                                              \
    }                                                                             \
    catch (const std::bad_alloc&) { return fail(handle, SB_EINTERNAL, "out of host memory"); } \
    catch (...) { return fail(handle, SB_EINTERNAL, "unexpected C++ exception"); }

// ---- GEMV argument checks shared by sb_gemv and sb_gemv_noalloc ----------

namespace {

struct GemvCall {
    sb_status st;
    bool empty;          // nothing to read or write
    sb_dtype dtype;
    bool row_dot;        // kernel N on the row-major view, else kernel T
    int64_t rows, cols;  // the row-major view
};

GemvCall check_gemv(const char* fn, sb_handle* handle, sb_dtype dtype, sb_layout layout, sb_op op, int64_t m,
                    int64_t n, const void* A, int64_t lda, const void* x, void* c)
{
    GemvCall g{SB_OK, false, dtype, false, 0, 0};
    auto bad = [&](sb_status st) { g.st = st; return g; };
    if (narrow(dtype)) return bad(fail(handle, SB_EUNSUPPORTED, "%s: narrow storage needs sb_gemv_q", fn));
    if (dtype != SB_F64 && dtype != SB_F32) return bad(fail(handle, SB_EINVAL, "%s: bad dtype %d", fn, (int)dtype));
    if (layout != SB_ROW_MAJOR && layout != SB_COL_MAJOR)
        return bad(fail(handle, SB_EINVAL, "%s: bad layout %d", fn, (int)layout));
    if (op != SB_N && op != SB_T) return bad(fail(handle, SB_EINVAL, "%s: bad op %d", fn, (int)op));
    if (m < 0 || n < 0)
        return bad(fail(handle, SB_EINVAL, "%s: negative size m=%lld n=%lld", fn, (long long)m, (long long)n));
    g.rows = layout == SB_ROW_MAJOR ? m : n;
    g.cols = layout == SB_ROW_MAJOR ? n : m;
    if (lda < (g.cols > 1 ? g.cols : 1))
        return bad(fail(handle, SB_EINVAL, "%s: lda=%lld below %lld", fn, (long long)lda,
                        (long long)(g.cols > 1 ? g.cols : 1)));
    const int es = esize_of(dtype);
    const int64_t a_el = span_elems(g.rows, g.cols, lda);
    int64_t a_bytes;
    if (a_el < 0 || !mul_ok(a_el, es, &a_bytes) || a_bytes > kMaxBytes)
        return bad(fail(handle, SB_EINVAL, "%s: matrix extent overflows", fn));
    const int64_t lx = op == SB_N ? n : m, lc = op == SB_N ? m : n;
    g.row_dot = (layout == SB_ROW_MAJOR) == (op == SB_N);
    // An empty output or an empty reduction reads and writes nothing.
    if (lc == 0 || lx == 0) {
        g.empty = true;
        return g;
    }
    if (!A || !x || !c) return bad(fail(handle, SB_EINVAL, "%s: NULL pointer with non-zero extent", fn));
    if (misaligned(A, es) || misaligned(x, es) || misaligned(c, es))
        return bad(fail(handle, SB_EINVAL, "%s: pointer not aligned to the element size", fn));
    const Range rc = range_of(c, lc, es);
    if (overlap(rc, range_of(A, a_el, es)) || overlap(rc, range_of(x, lx, es)))
        return bad(fail(handle, SB_EINVAL, "%s: c overlaps A or x", fn));
    return g;
}

// Workspace bytes of a checked, non-empty GEMV with the handle's tuning.
size_t gemv_ws_bytes(const sb_handle* handle, const GemvCall& g)
{
    const int es = esize_of(g.dtype);
    return g.row_dot ? sb::plan_gemv_n(es, g.rows, g.cols).ws
                     : sb::plan_gemv_t(es, g.rows, g.cols, handle->gemv_t_small_splits).ws;
}

sb_status run_checked_gemv(sb_handle* h, const GemvCall& g, const void* A, int64_t lda, const void* x, void* c)
{
    return g.row_dot ? sb::run_gemv_n(h, g.dtype, g.rows, g.cols, A, lda, x, c)
                     : sb::run_gemv_t(h, g.dtype, g.rows, g.cols, A, lda, x, c);
}

// ---- the static scratch of sb_gemv_noalloc -------------------------------
//
// One array per GPU in this library's device code, used by sb_gemv_noalloc
// in place of a workspace.  In host code the name `noalloc_scratch_array`
// is only a host-side stand-in: its device address is looked up once per
// device with hipGetSymbolAddress (with that device current) and only that
// address is ever handed to kernels.

constexpr size_t kNoAllocScratchBytes = SB_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char noalloc_scratch_array[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of the scratch on the device of the handle's stream.
sb_status noalloc_scratch(sb_handle* h, void** out)
{
    int dev = -1, cur = -1;
    hipError_t e = hipStreamGetDevice(h->stream, &dev);
    if (e != hipSuccess) return fail(h, SB_EDEVICE, "sb_gemv_noalloc: hipStreamGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(h, SB_EDEVICE, "sb_gemv_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch_array));
        const hipError_t e_restore = (cur >= 0 && cur != dev) ? hipSetDevice(cur) : hipSuccess;
        if (e != hipSuccess)
            return fail(h, SB_EDEVICE, "sb_gemv_noalloc: scratch address on device %d: %s", dev, hipGetErrorString(e));
        if (e_restore != hipSuccess)
            return fail(h, SB_EDEVICE, "sb_gemv_noalloc: restoring device %d: %s", cur, hipGetErrorString(e_restore));
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return SB_OK;
}

}  // namespace

extern "C" {

int32_t sb_version(void) { return 100; }

const char* sb_status_string(sb_status status)
{
    if (status > 0 || status < SB_EINTERNAL) return "unknown status";
    return kStatusText[-status];
}

sb_status sb_handle_create(void* workspace, size_t ws_bytes, void* stream, sb_handle** out)
{
    if (!out) return fail(nullptr, SB_EINVAL, "sb_handle_create: out is NULL");
    *out = nullptr;
    if (!workspace && ws_bytes) return fail(nullptr, SB_EINVAL, "sb_handle_create: NULL workspace of %zu bytes", ws_bytes);
    sb_handle* h = new (std::nothrow) sb_handle;
    if (!h) return fail(nullptr, SB_EINTERNAL, "sb_handle_create: out of host memory");
    h->ws = workspace;
    h->ws_bytes = workspace ? ws_bytes : 0;
    h->ws_gen = 0;
    h->stream = static_cast<hipStream_t>(stream);
    h->dot_small_bytes = sb::kDefaultDotSmallBytes;
    h->gemv_t_small_splits = sb::kDefaultGemvTSmallSplits;
    h->err[0] = '\0';
    *out = h;
    return SB_OK;
}

sb_status sb_handle_destroy(sb_handle* handle)
{
    delete handle;
    return SB_OK;
}

sb_status sb_set_stream(sb_handle* handle, void* stream)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_set_stream: NULL handle");
    handle->stream = static_cast<hipStream_t>(stream);
    return SB_OK;
}

sb_status sb_set_workspace(sb_handle* handle, void* workspace, size_t ws_bytes)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_set_workspace: NULL handle");
    if (!workspace && ws_bytes) return fail(handle, SB_EINVAL, "sb_set_workspace: NULL workspace of %zu bytes", ws_bytes);
    handle->ws = workspace;
    handle->ws_bytes = workspace ? ws_bytes : 0;
    ++handle->ws_gen;
    return SB_OK;
}

sb_status sb_set_cutoff(sb_handle* handle, sb_cutoff which, int64_t value)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_set_cutoff: NULL handle");
    if (value < 0) return fail(handle, SB_EINVAL, "sb_set_cutoff: negative value %lld", (long long)value);
    switch (which) {
    case SB_CUTOFF_DOT_SMALL_BYTES: handle->dot_small_bytes = value; return SB_OK;
    case SB_CUTOFF_GEMV_T_SMALL_SPLITS: handle->gemv_t_small_splits = value; return SB_OK;
    }
    return fail(handle, SB_EINVAL, "sb_set_cutoff: unknown cutoff %d", (int)which);
}

sb_status sb_get_cutoff(const sb_handle* handle, sb_cutoff which, int64_t* value)
{
    if (!value) return fail(nullptr, SB_EINVAL, "sb_get_cutoff: value is NULL");
    switch (which) {
    case SB_CUTOFF_DOT_SMALL_BYTES:
        *value = handle ? handle->dot_small_bytes : sb::kDefaultDotSmallBytes;
        return SB_OK;
    case SB_CUTOFF_GEMV_T_SMALL_SPLITS:
        *value = handle ? handle->gemv_t_small_splits : sb::kDefaultGemvTSmallSplits;
        return SB_OK;
    }
    return fail(nullptr, SB_EINVAL, "sb_get_cutoff: unknown cutoff %d", (int)which);
}

const char* sb_last_error(const sb_handle* handle) { return handle ? handle->err : g_err; }

size_t sb_workspace_bytes(const sb_handle* handle, sb_kind kind, sb_dtype dtype, sb_layout layout,
                          sb_op op, int64_t m, int64_t n)
{
    const int64_t dot_small = handle ? handle->dot_small_bytes : sb::kDefaultDotSmallBytes;
    const int64_t t_small = handle ? handle->gemv_t_small_splits : sb::kDefaultGemvTSmallSplits;
    const size_t bad = (size_t)-1;
    if (m < 0 || n < 0) return bad;
    switch (kind) {
    case SB_KIND_GEMV: {
        if (dtype != SB_F64 && dtype != SB_F32) return bad;
        if ((layout != SB_ROW_MAJOR && layout != SB_COL_MAJOR) || (op != SB_N && op != SB_T)) return bad;
        if (m == 0 || n == 0) return 0;
        const int es = esize_of(dtype);
        const int64_t rows = layout == SB_ROW_MAJOR ? m : n, cols = layout == SB_ROW_MAJOR ? n : m;
        const bool row_dot = (layout == SB_ROW_MAJOR) == (op == SB_N);
        return row_dot ? sb::plan_gemv_n(es, rows, cols).ws : sb::plan_gemv_t(es, rows, cols, t_small).ws;
    }
    case SB_KIND_GEMV_MX:
        if (!is_mx(dtype)) return bad;
        return (m == 0 || n == 0) ? 0 : sb::gemv_mx_ws_bytes(dtype, m, n);
    case SB_KIND_GEMV2: {
        if (dtype != SB_F64 && dtype != SB_F32) return bad;
        if (layout != SB_ROW_MAJOR && layout != SB_COL_MAJOR) return bad;
        if (m == 0 || n == 0) return 0;
        const int64_t rows = layout == SB_ROW_MAJOR ? m : n, cols = layout == SB_ROW_MAJOR ? n : m;
        return sb::plan_gemv2(esize_of(dtype), rows, cols).ws;
    }
    case SB_KIND_DOT:
        if (dtype != SB_F64 && dtype != SB_F32) return bad;
        return n == 0 ? 0 : sb::plan_dot(esize_of(dtype), n, 1, dot_small).ws;
    case SB_KIND_DOT2:
        return n == 0 ? 0 : sb::plan_dot(4, n, 2, dot_small).ws;
    case SB_KIND_GEMV_Q:
        if (dtype != SB_BF16 && dtype != SB_FP8_E4M3) return bad;
        return (m == 0 || n == 0) ? 0 : sb::gemv_q_ws_bytes(dtype, m, n);
    case SB_KIND_GER:
        return 0;
    case SB_KIND_PROBE_READ:
        return sb::probe_ws_bytes((size_t)n);
    }
    return bad;
}

sb_status sb_gemv(sb_handle* handle, sb_dtype dtype, sb_layout layout, sb_op op, int64_t m, int64_t n,
                  const void* A, int64_t lda, const void* x, void* c)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_gemv: NULL handle");
    SB_GUARD_BEGIN
    const GemvCall g = check_gemv("sb_gemv", handle, dtype, layout, op, m, n, A, lda, x, c);
    if (g.st != SB_OK || g.empty) return g.st;
    return run_checked_gemv(handle, g, A, lda, x, c);
    SB_GUARD_END
}

sb_status sb_gemv_noalloc(sb_handle* handle, sb_dtype dtype, sb_layout layout, sb_op op, int64_t m, int64_t n,
                          const void* A, int64_t lda, const void* x, void* c)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_gemv_noalloc: NULL handle");
    SB_GUARD_BEGIN
    const GemvCall g = check_gemv("sb_gemv_noalloc", handle, dtype, layout, op, m, n, A, lda, x, c);
    if (g.st != SB_OK || g.empty) return g.st;
    const size_t need = gemv_ws_bytes(handle, g);
    if (need > kNoAllocScratchBytes)
        return fail(handle, SB_ENOMEM,
                    "sb_gemv_noalloc: this shape needs %zu bytes of split partial sums; the static scratch holds %zu",
                    need, (size_t)kNoAllocScratchBytes);
    // The same call on a copy of the handle whose workspace is this device's
    // static scratch: the caller's workspace (and any plan in it) is untouched.
    sb_handle view = *handle;
    if (need > 0) {
        void* p = nullptr;
        const sb_status st = noalloc_scratch(handle, &p);
        if (st != SB_OK) return st;
        view.ws = p;
        view.ws_bytes = kNoAllocScratchBytes;
    } else {
        view.ws = nullptr;
        view.ws_bytes = 0;
    }
    const sb_status st = run_checked_gemv(&view, g, A, lda, x, c);
    if (st != SB_OK) memcpy(handle->err, view.err, sizeof(handle->err));
    return st;
    SB_GUARD_END
}

sb_status sb_gemv2(sb_handle* handle, sb_dtype dtype, sb_layout layout, int64_t m, int64_t n, const void* A,
                   int64_t lda, const void* x, const void* y, void* c, void* d)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_gemv2: NULL handle");
    SB_GUARD_BEGIN
    if (narrow(dtype)) return fail(handle, SB_EUNSUPPORTED, "sb_gemv2: narrow dtype");
    if (dtype != SB_F64 && dtype != SB_F32) return fail(handle, SB_EINVAL, "sb_gemv2: bad dtype %d", (int)dtype);
    if (layout != SB_ROW_MAJOR && layout != SB_COL_MAJOR) return fail(handle, SB_EINVAL, "sb_gemv2: bad layout %d", (int)layout);
    if (m < 0 || n < 0) return fail(handle, SB_EINVAL, "sb_gemv2: negative size m=%lld n=%lld", (long long)m, (long long)n);
    const int64_t rows = layout == SB_ROW_MAJOR ? m : n, cols = layout == SB_ROW_MAJOR ? n : m;
    if (lda < (cols > 1 ? cols : 1))
        return fail(handle, SB_EINVAL, "sb_gemv2: lda=%lld below %lld", (long long)lda, (long long)(cols > 1 ? cols : 1));
    const int es = esize_of(dtype);
    const int64_t a_el = span_elems(rows, cols, lda);
    int64_t a_bytes;
    if (a_el < 0 || !mul_ok(a_el, es, &a_bytes) || a_bytes > kMaxBytes)
        return fail(handle, SB_EINVAL, "sb_gemv2: matrix extent overflows");
    if (m == 0 || n == 0) return SB_OK;
    if (!A || !x || !y || !c || !d) return fail(handle, SB_EINVAL, "sb_gemv2: NULL pointer with non-zero extent");
    if (misaligned(A, es) || misaligned(x, es) || misaligned(y, es) || misaligned(c, es) || misaligned(d, es))
        return fail(handle, SB_EINVAL, "sb_gemv2: pointer not aligned to the element size");
    const Range ra = range_of(A, a_el, es), rx = range_of(x, n, es), ry = range_of(y, m, es);
    const Range rc = range_of(c, m, es), rd = range_of(d, n, es);
    if (overlap(rc, ra) || overlap(rc, rx) || overlap(rc, ry) || overlap(rd, ra) || overlap(rd, rx) ||
        overlap(rd, ry) || overlap(rc, rd))
        return fail(handle, SB_EINVAL, "sb_gemv2: c or d overlaps A, x, y or the other output");
    // On the row-major view: row-dot gives c (row-major) or d (column-major).
    if (layout == SB_ROW_MAJOR) return sb::run_gemv2(handle, dtype, rows, cols, A, lda, x, y, c, d);
    return sb::run_gemv2(handle, dtype, rows, cols, A, lda, y, x, d, c);
    SB_GUARD_END
}

sb_status sb_dot(sb_handle* handle, sb_dtype dtype, int64_t n, const void* x, const void* y, void* alpha)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_dot: NULL handle");
    SB_GUARD_BEGIN
    if (narrow(dtype)) return fail(handle, SB_EUNSUPPORTED, "sb_dot: narrow dtype");
    if (dtype != SB_F64 && dtype != SB_F32) return fail(handle, SB_EINVAL, "sb_dot: bad dtype %d", (int)dtype);
    if (n < 0) return fail(handle, SB_EINVAL, "sb_dot: negative n=%lld", (long long)n);
    const int es = esize_of(dtype);
    int64_t bytes;
    if (!mul_ok(n, es, &bytes) || bytes > kMaxBytes) return fail(handle, SB_EINVAL, "sb_dot: n overflows");
    if (!alpha || (n > 0 && (!x || !y))) return fail(handle, SB_EINVAL, "sb_dot: NULL pointer");
    if (misaligned(x, es) || misaligned(y, es) || misaligned(alpha, es))
        return fail(handle, SB_EINVAL, "sb_dot: pointer not aligned to the element size");
    const Range ra = range_of(alpha, 1, es);
    if (overlap(ra, range_of(x, n, es)) || overlap(ra, range_of(y, n, es)))
        return fail(handle, SB_EINVAL, "sb_dot: alpha overlaps x or y");
    return sb::run_dot(handle, dtype, n, x, y, alpha);
    SB_GUARD_END
}

sb_status sb_ger(sb_handle* handle, sb_dtype dtype, sb_layout layout, int64_t m, int64_t n, const void* x,
                 const void* y, void* C, int64_t ldc)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_ger: NULL handle");
    SB_GUARD_BEGIN
    if (narrow(dtype)) return fail(handle, SB_EUNSUPPORTED, "sb_ger: narrow dtype");
    if (dtype != SB_F64 && dtype != SB_F32) return fail(handle, SB_EINVAL, "sb_ger: bad dtype %d", (int)dtype);
    if (layout != SB_ROW_MAJOR && layout != SB_COL_MAJOR) return fail(handle, SB_EINVAL, "sb_ger: bad layout %d", (int)layout);
    if (m < 0 || n < 0) return fail(handle, SB_EINVAL, "sb_ger: negative size");
    const int64_t rows = layout == SB_ROW_MAJOR ? m : n, cols = layout == SB_ROW_MAJOR ? n : m;
    if (ldc < (cols > 1 ? cols : 1)) return fail(handle, SB_EINVAL, "sb_ger: ldc=%lld too small", (long long)ldc);
    const int es = esize_of(dtype);
    const int64_t c_el = span_elems(rows, cols, ldc);
    int64_t c_bytes;
    if (c_el < 0 || !mul_ok(c_el, es, &c_bytes) || c_bytes > kMaxBytes)
        return fail(handle, SB_EINVAL, "sb_ger: matrix extent overflows");
    if ((c_el > 0 && (!C || !x || !y))) return fail(handle, SB_EINVAL, "sb_ger: NULL pointer with non-zero extent");
    if (misaligned(x, es) || misaligned(y, es) || misaligned(C, es))
        return fail(handle, SB_EINVAL, "sb_ger: pointer not aligned to the element size");
    const Range rC = range_of(C, c_el, es);
    if (overlap(rC, range_of(x, m, es)) || overlap(rC, range_of(y, n, es)))
        return fail(handle, SB_EINVAL, "sb_ger: C overlaps x or y");
    if (c_el == 0) return SB_OK;
    if (layout == SB_ROW_MAJOR) return sb::run_ger(handle, dtype, m, n, x, y, C, ldc);
    return sb::run_ger(handle, dtype, n, m, y, x, C, ldc);
    SB_GUARD_END
}

sb_status sb_quantize_rows(sb_handle* handle, sb_dtype q, int64_t m, int64_t n, const float* A, int64_t lda,
                           void* Aq, int64_t ldq, float* scales)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_quantize_rows: NULL handle");
    SB_GUARD_BEGIN
    if (q != SB_BF16 && q != SB_FP8_E4M3) return fail(handle, SB_EINVAL, "sb_quantize_rows: q must be BF16 or FP8_E4M3");
    if (m < 0 || n < 0) return fail(handle, SB_EINVAL, "sb_quantize_rows: negative size");
    const int64_t need = n > 1 ? n : 1;
    if (lda < need || ldq < need) return fail(handle, SB_EINVAL, "sb_quantize_rows: lda/ldq below n");
    const int qs = esize_of(q);
    const int64_t a_el = span_elems(m, n, lda), q_el = span_elems(m, n, ldq);
    int64_t t, tq;
    if (a_el < 0 || q_el < 0 || !mul_ok(a_el, 4, &t) || t > kMaxBytes || !mul_ok(q_el, qs, &tq) || tq > kMaxBytes)
        return fail(handle, SB_EINVAL, "sb_quantize_rows: extent overflows");
    if ((a_el > 0 && (!A || !Aq)) || (m > 0 && !scales)) return fail(handle, SB_EINVAL, "sb_quantize_rows: NULL pointer");
    if (misaligned(A, 4) || misaligned(Aq, qs) || misaligned(scales, 4))
        return fail(handle, SB_EINVAL, "sb_quantize_rows: pointer not aligned to the element size");
    const Range rq = range_of(Aq, q_el, qs), rs = range_of(scales, m, 4), ra = range_of(A, a_el, 4);
    if (overlap(rq, ra) || overlap(rs, ra) || overlap(rs, rq))
        return fail(handle, SB_EINVAL, "sb_quantize_rows: outputs overlap");
    return sb::run_quantize_rows(handle, q, m, n, A, lda, Aq, ldq, scales);
    SB_GUARD_END
}

sb_status sb_gemv_q(sb_handle* handle, sb_dtype q, int64_t m, int64_t n, const void* Aq, int64_t ldq,
                    const float* scales, const float* x, float* c)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_gemv_q: NULL handle");
    SB_GUARD_BEGIN
    if (q != SB_BF16 && q != SB_FP8_E4M3) return fail(handle, SB_EINVAL, "sb_gemv_q: q must be BF16 or FP8_E4M3");
    if (m < 0 || n < 0) return fail(handle, SB_EINVAL, "sb_gemv_q: negative size");
    if (ldq < (n > 1 ? n : 1)) return fail(handle, SB_EINVAL, "sb_gemv_q: ldq below n");
    const int qs = esize_of(q);
    const int64_t q_el = span_elems(m, n, ldq);
    int64_t t;
    if (q_el < 0 || !mul_ok(q_el, qs, &t) || t > kMaxBytes) return fail(handle, SB_EINVAL, "sb_gemv_q: extent overflows");
    if ((q_el > 0 && (!Aq || !x)) || (m > 0 && (!scales || !c))) return fail(handle, SB_EINVAL, "sb_gemv_q: NULL pointer");
    if (misaligned(Aq, qs) || misaligned(scales, 4) || misaligned(x, 4) || misaligned(c, 4))
        return fail(handle, SB_EINVAL, "sb_gemv_q: pointer not aligned to the element size");
    const Range rc = range_of(c, m, 4);
    if (overlap(rc, range_of(Aq, q_el, qs)) || overlap(rc, range_of(scales, m, 4)) || overlap(rc, range_of(x, n, 4)))
        return fail(handle, SB_EINVAL, "sb_gemv_q: c overlaps an input");
    return sb::run_gemv_q(handle, q, m, n, Aq, ldq, scales, x, c);
    SB_GUARD_END
}

// Checks shared by the MX quantiser and GEMV: sizes, strides, extents.
static sb_status mx_layout_check(sb_handle* handle, const char* what, sb_dtype q, int64_t m, int64_t n, int64_t ldq,
                                 int64_t lds, int64_t* q_bytes, int64_t* s_bytes)
{
    if (!is_mx(q)) return fail(handle, SB_EINVAL, "%s: q must be MXFP8_E4M3 or MXFP4_E2M1", what);
    if (m < 0 || n < 0) return fail(handle, SB_EINVAL, "%s: negative size", what);
    const int64_t rb = mx_row_bytes(q, n), nb = (n + 31) / 32;
    if (ldq < (rb > 1 ? rb : 1) || ldq % 16 != 0)
        return fail(handle, SB_EINVAL, "%s: ldq=%lld must cover a row (%lld bytes) and be a multiple of 16", what,
                    (long long)ldq, (long long)rb);
    if (lds < (nb > 1 ? nb : 1)) return fail(handle, SB_EINVAL, "%s: lds=%lld below %lld blocks", what, (long long)lds, (long long)nb);
    *q_bytes = span_elems(m, rb, ldq);
    *s_bytes = span_elems(m, nb, lds);
    if (*q_bytes < 0 || *s_bytes < 0 || *q_bytes > kMaxBytes || *s_bytes > kMaxBytes)
        return fail(handle, SB_EINVAL, "%s: extent overflows", what);
    return SB_OK;
}

sb_status sb_quantize_mx(sb_handle* handle, sb_dtype q, int64_t m, int64_t n, const float* A, int64_t lda, void* Q,
                         int64_t ldq, uint8_t* S, int64_t lds)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_quantize_mx: NULL handle");
    SB_GUARD_BEGIN
    int64_t qb, sbytes;
    sb_status st = mx_layout_check(handle, "sb_quantize_mx", q, m, n, ldq, lds, &qb, &sbytes);
    if (st != SB_OK) return st;
    if (lda < (n > 1 ? n : 1)) return fail(handle, SB_EINVAL, "sb_quantize_mx: lda below n");
    const int64_t a_el = span_elems(m, n, lda);
    int64_t t;
    if (a_el < 0 || !mul_ok(a_el, 4, &t) || t > kMaxBytes) return fail(handle, SB_EINVAL, "sb_quantize_mx: extent overflows");
    if (m == 0 || n == 0) return SB_OK;
    if (!A || !Q || !S) return fail(handle, SB_EINVAL, "sb_quantize_mx: NULL pointer");
    if (misaligned(A, 4) || (reinterpret_cast<uintptr_t>(Q) & 15u) != 0)
        return fail(handle, SB_EINVAL, "sb_quantize_mx: A must be 4-byte and Q 16-byte aligned");
    const Range ra = range_of(A, a_el, 4), rq = range_of(Q, qb, 1), rs = range_of(S, sbytes, 1);
    if (overlap(ra, rq) || overlap(ra, rs) || overlap(rq, rs))
        return fail(handle, SB_EINVAL, "sb_quantize_mx: A, Q and S must not overlap");
    return sb::run_quantize_mx(handle, q, m, n, A, lda, Q, ldq, S, lds);
    SB_GUARD_END
}

sb_status sb_gemv_mx(sb_handle* handle, sb_dtype q, int64_t m, int64_t n, const void* Q, int64_t ldq,
                     const uint8_t* S, int64_t lds, const float* x, float* c)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_gemv_mx: NULL handle");
    SB_GUARD_BEGIN
    int64_t qb, sbytes;
    sb_status st = mx_layout_check(handle, "sb_gemv_mx", q, m, n, ldq, lds, &qb, &sbytes);
    if (st != SB_OK) return st;
    if (m == 0 || n == 0) return SB_OK;
    if (!Q || !S || !x || !c) return fail(handle, SB_EINVAL, "sb_gemv_mx: NULL pointer");
    if ((reinterpret_cast<uintptr_t>(Q) & 15u) != 0 || misaligned(x, 4) || misaligned(c, 4))
        return fail(handle, SB_EINVAL, "sb_gemv_mx: Q must be 16-byte and x, c 4-byte aligned");
    const Range rc = range_of(c, m, 4);
    if (overlap(rc, range_of(Q, qb, 1)) || overlap(rc, range_of(S, sbytes, 1)) || overlap(rc, range_of(x, n, 4)))
        return fail(handle, SB_EINVAL, "sb_gemv_mx: c overlaps an input");
    return sb::run_gemv_mx(handle, q, m, n, Q, ldq, S, lds, x, c);
    SB_GUARD_END
}

sb_status sb_dot2_f32(sb_handle* handle, int64_t n, const float* x, const float* y, float* alpha)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_dot2_f32: NULL handle");
    SB_GUARD_BEGIN
    if (n < 0) return fail(handle, SB_EINVAL, "sb_dot2_f32: negative n");
    int64_t bytes;
    if (!mul_ok(n, 4, &bytes) || bytes > kMaxBytes) return fail(handle, SB_EINVAL, "sb_dot2_f32: n overflows");
    if (!alpha || (n > 0 && (!x || !y))) return fail(handle, SB_EINVAL, "sb_dot2_f32: NULL pointer");
    if (misaligned(x, 4) || misaligned(y, 4) || misaligned(alpha, 4))
        return fail(handle, SB_EINVAL, "sb_dot2_f32: pointer not aligned to the element size");
    const Range ra = range_of(alpha, 1, 4);
    if (overlap(ra, range_of(x, n, 4)) || overlap(ra, range_of(y, n, 4)))
        return fail(handle, SB_EINVAL, "sb_dot2_f32: alpha overlaps x or y");
    return sb::run_dot2(handle, n, x, y, alpha);
    SB_GUARD_END
}

sb_status sb_fill_uniform(sb_handle* handle, sb_dtype dtype, void* out, int64_t count, uint64_t seed,
                          uint64_t counter0)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_fill_uniform: NULL handle");
    if (dtype != SB_F64 && dtype != SB_F32) return fail(handle, SB_EINVAL, "sb_fill_uniform: dtype must be F64 or F32");
    if (count < 0 || count > kMaxBytes / 8) return fail(handle, SB_EINVAL, "sb_fill_uniform: bad count");
    if (count > 0 && (!out || misaligned(out, esize_of(dtype))))
        return fail(handle, SB_EINVAL, "sb_fill_uniform: NULL or misaligned output");
    if (dtype == SB_F32 && count > 0 && counter0 > ~(uint64_t)0 - (uint64_t)(count - 1))
        return fail(handle, SB_EINVAL, "sb_fill_uniform: binary32 counters counter0 .. counter0 + count - 1 wrap past 2^64");
    SB_GUARD_BEGIN
    return sb::run_fill_uniform(handle, dtype, out, count, seed, counter0);
    SB_GUARD_END
}

static sb_status probe_check(sb_handle* handle, const char* what, const void* src, const void* dst, size_t bytes)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "%s: NULL handle", what);
    if (bytes % 16) return fail(handle, SB_EINVAL, "%s: bytes must be a multiple of 16", what);
    if (bytes > (size_t)kMaxBytes) return fail(handle, SB_EINVAL, "%s: size too large", what);
    if (bytes && (!src || !sb::aligned16(src) || (dst && !sb::aligned16(dst))))
        return fail(handle, SB_EINVAL, "%s: NULL or misaligned pointer", what);
    if (dst && overlap(range_of(src, (int64_t)bytes, 1), range_of(dst, (int64_t)bytes, 1)))
        return fail(handle, SB_EINVAL, "%s: ranges overlap", what);
    return SB_OK;
}

sb_status sb_stream_read(sb_handle* handle, const void* src, size_t bytes)
{
    sb_status st = probe_check(handle, "sb_stream_read", src, nullptr, bytes);
    if (st != SB_OK) return st;
    SB_GUARD_BEGIN
    return sb::run_stream_read(handle, src, bytes);
    SB_GUARD_END
}

sb_status sb_stream_copy(sb_handle* handle, const void* src, void* dst, size_t bytes)
{
    if (bytes && !dst) return fail(handle, SB_EINVAL, "sb_stream_copy: NULL destination");
    sb_status st = probe_check(handle, "sb_stream_copy", src, dst, bytes);
    if (st != SB_OK) return st;
    SB_GUARD_BEGIN
    return sb::run_stream_copy(handle, src, dst, bytes);
    SB_GUARD_END
}

sb_status sb_stream_update(sb_handle* handle, void* C, int64_t rows, int64_t cols, int64_t ldc)
{
    if (!handle) return fail(nullptr, SB_EINVAL, "sb_stream_update: NULL handle");
    if (rows < 0 || cols < 0 || ldc < (cols > 1 ? cols : 1))
        return fail(handle, SB_EINVAL, "sb_stream_update: bad size or leading dimension");
    const int64_t el = span_elems(rows, cols, ldc);
    int64_t bytes;
    if (el < 0 || !mul_ok(el, 8, &bytes) || bytes > kMaxBytes)
        return fail(handle, SB_EINVAL, "sb_stream_update: extent overflows");
    if (rows == 0 || cols == 0) return SB_OK;
    if (!C || misaligned(C, 8)) return fail(handle, SB_EINVAL, "sb_stream_update: NULL or misaligned matrix");
    SB_GUARD_BEGIN
    return sb::run_stream_update(handle, C, rows, cols, ldc);
    SB_GUARD_END
}

}  // extern "C"
