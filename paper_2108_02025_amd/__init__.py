"""Python binding of streamblas (``libstreamblas.so``, declared in
``include/streamblas.h``): GEMV, DOT and GER of Singh and Bassoy, "High
Performance Level-1 and Level-2 BLAS" (arXiv 2108.02025, section 3.1
definitions), on one MI355X.

The functions carry the C names and only marshal arguments: they read
pointers, sizes and strides from torch tensors, pick the handle of the
tensor's device, size its workspace and pass the current torch stream.  All
arithmetic runs in the library's HIP kernels.  There is no fallback: if the
library is not built, ``load()`` raises.

torch is imported first on purpose: the library links the HIP runtime that
torch loads, so one process holds one runtime.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "SB_F64", "SB_F32", "SB_BF16", "SB_FP8_E4M3", "SB_ROW_MAJOR", "SB_COL_MAJOR", "SB_N", "SB_T",
    "SB_KIND_GEMV", "SB_KIND_DOT", "SB_KIND_GER", "SB_KIND_GEMV_Q", "SB_KIND_DOT2", "SB_KIND_GEMV2", "sb_gemv2",
    "StreamBlasError", "load", "lib_path", "Handle", "handle_for",
    "sb_version", "sb_status_string", "sb_workspace_bytes",
    "sb_gemv", "sb_gemv_noalloc", "sb_dot", "sb_ger", "sb_quantize_rows", "sb_gemv_q", "sb_dot2_f32",
    "sb_stream_read", "sb_stream_copy", "sb_stream_update", "sb_gemv_desc", "GemvProblem", "make_descs", "sb_gemv_batched",
    "sb_gemv_batched_resolve", "sb_gemv_batched_table_bytes", "BatchTable", "sb_fill_uniform",
    "SB_CUTOFF_DOT_SMALL_BYTES", "SB_CUTOFF_GEMV_T_SMALL_SPLITS", "sb_set_cutoff", "sb_get_cutoff",
    "SB_MXFP8_E4M3", "SB_MXFP4_E2M1", "SB_KIND_GEMV_MX", "mx_buffers", "sb_quantize_mx", "sb_gemv_mx",
    "Plan",
]

SB_OK, SB_EINVAL, SB_ENOMEM, SB_EDEVICE, SB_EUNSUPPORTED, SB_EINTERNAL = 0, -1, -2, -3, -4, -5
SB_F64, SB_F32, SB_BF16, SB_FP8_E4M3, SB_MXFP8_E4M3, SB_MXFP4_E2M1 = 0, 1, 2, 3, 4, 5
SB_ROW_MAJOR, SB_COL_MAJOR = 0, 1
SB_N, SB_T = 0, 1
SB_KIND_GEMV, SB_KIND_DOT, SB_KIND_GER, SB_KIND_GEMV_Q, SB_KIND_DOT2, SB_KIND_PROBE_READ = 0, 1, 2, 3, 4, 5
SB_KIND_GEMV2, SB_KIND_GEMV_MX = 6, 7
SB_CUTOFF_DOT_SMALL_BYTES, SB_CUTOFF_GEMV_T_SMALL_SPLITS = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libstreamblas.so")

_DTYPES = {torch.float64: SB_F64, torch.float32: SB_F32}


class sb_gemv_desc(ctypes.Structure):
    """One problem of a batched GEMV (layout of the C struct)."""
    _fields_ = [("dtype", ctypes.c_int32), ("group", ctypes.c_int32), ("rows_per_tile", ctypes.c_int32),
                ("split", ctypes.c_int32), ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("x", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("layout", ctypes.c_int32), ("op", ctypes.c_int32)]


class StreamBlasError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libstreamblas.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(lib_path):
        raise FileNotFoundError(f"{lib_path} is not built; run python -m paper_2108_02025_amd.build")
    L = ctypes.CDLL(lib_path)
    P, I64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    L.sb_version.restype = I32
    L.sb_status_string.argtypes = [I32]
    L.sb_status_string.restype = ctypes.c_char_p
    L.sb_handle_create.argtypes = [P, SZ, P, ctypes.POINTER(P)]
    L.sb_handle_destroy.argtypes = [P]
    L.sb_set_stream.argtypes = [P, P]
    L.sb_set_workspace.argtypes = [P, P, SZ]
    L.sb_last_error.argtypes = [P]
    L.sb_last_error.restype = ctypes.c_char_p
    L.sb_set_cutoff.argtypes = [P, I32, I64]
    L.sb_get_cutoff.argtypes = [P, I32, ctypes.POINTER(I64)]
    L.sb_workspace_bytes.argtypes = [P, I32, I32, I32, I32, I64, I64]
    L.sb_workspace_bytes.restype = SZ
    L.sb_gemv.argtypes = [P, I32, I32, I32, I64, I64, P, I64, P, P]
    L.sb_gemv_noalloc.argtypes = [P, I32, I32, I32, I64, I64, P, I64, P, P]
    L.sb_dot.argtypes = [P, I32, I64, P, P, P]
    L.sb_gemv2.argtypes = [P, I32, I32, I64, I64, P, I64, P, P, P, P]
    L.sb_ger.argtypes = [P, I32, I32, I64, I64, P, P, P, I64]
    L.sb_quantize_rows.argtypes = [P, I32, I64, I64, P, I64, P, I64, P]
    L.sb_gemv_q.argtypes = [P, I32, I64, I64, P, I64, P, P, P]
    L.sb_dot2_f32.argtypes = [P, I64, P, P, P]
    L.sb_quantize_mx.argtypes = [P, I32, I64, I64, P, I64, P, I64, P, I64]
    L.sb_gemv_mx.argtypes = [P, I32, I64, I64, P, I64, P, I64, P, P]
    L.sb_gemv_batched_table_bytes.argtypes = [ctypes.POINTER(sb_gemv_desc), I32, ctypes.POINTER(SZ)]
    L.sb_gemv_batched_table_bytes.restype = SZ
    L.sb_gemv_batched_resolve.argtypes = [ctypes.POINTER(sb_gemv_desc), I32, ctypes.POINTER(sb_gemv_desc)]
    L.sb_gemv_batched_encode.argtypes = [ctypes.POINTER(sb_gemv_desc), I32, P, P, SZ]
    L.sb_gemv_batched_run.argtypes = [P, P, I32]
    L.sb_gemv_batched.argtypes = [P, ctypes.POINTER(sb_gemv_desc), I32]
    L.sb_plan_create.argtypes = [P, ctypes.POINTER(sb_gemv_desc), I32, ctypes.POINTER(P)]
    L.sb_plan_run.argtypes = [P]
    L.sb_plan_destroy.argtypes = [P]
    L.sb_fill_uniform.argtypes = [P, I32, P, I64, ctypes.c_uint64, ctypes.c_uint64]
    L.sb_generate_batched_bytes.argtypes = [I32]
    L.sb_generate_batched_bytes.restype = SZ
    L.sb_generate_batched.argtypes = [P, P, I32]
    L.sb_stream_read.argtypes = [P, P, SZ]
    L.sb_stream_copy.argtypes = [P, P, P, SZ]
    L.sb_stream_update.argtypes = [P, P, I64, I64, I64]
    for f in ("sb_fill_uniform", "sb_generate_batched", "sb_gemv_batched_resolve", "sb_gemv_batched_encode", "sb_gemv_batched_run", "sb_gemv_batched",
              "sb_stream_read", "sb_stream_copy", "sb_stream_update", "sb_handle_create", "sb_handle_destroy", "sb_set_stream", "sb_set_workspace", "sb_set_cutoff", "sb_get_cutoff", "sb_gemv", "sb_gemv_noalloc", "sb_gemv2",
              "sb_dot", "sb_ger", "sb_quantize_rows", "sb_gemv_q", "sb_dot2_f32", "sb_quantize_mx", "sb_gemv_mx",
              "sb_plan_create", "sb_plan_run", "sb_plan_destroy"):
        getattr(L, f).restype = I32
    _lib = L
    return L


def sb_version() -> int:
    return int(load().sb_version())


def sb_status_string(status: int) -> str:
    return load().sb_status_string(status).decode()


class Handle:
    """An sb_handle bound to one device, with a workspace owned by torch."""

    def __init__(self, device=None):
        L = load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self._ws = None
        h = ctypes.c_void_p()
        st = L.sb_handle_create(None, 0, None, ctypes.byref(h))
        if st != SB_OK:
            raise StreamBlasError(st, L.sb_last_error(None).decode())
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sb_handle_destroy(self.h)
            self.h = None

    def error(self) -> str:
        return load().sb_last_error(self.h).decode()

    def prepare(self, nbytes: int):
        """Point the handle at the current stream and a workspace of >= nbytes."""
        L = load()
        if nbytes == (1 << 64) - 1:
            raise StreamBlasError(SB_EINVAL, "invalid arguments for workspace sizing")
        if nbytes and (self._ws is None or self._ws.numel() < nbytes):
            self._ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            L.sb_set_workspace(self.h, ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel())
        L.sb_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def check(self, st: int):
        if st != SB_OK:
            raise StreamBlasError(st, self.error())


_handles: dict[int, Handle] = {}


def sb_get_cutoff(which: int, handle: Handle | None = None) -> int:
    """A handle's small-problem cutoff, or the library default (handle None)."""
    v = ctypes.c_int64()
    st = load().sb_get_cutoff(handle.h if handle else None, which, ctypes.byref(v))
    if st != SB_OK:
        raise StreamBlasError(st, load().sb_last_error(None).decode())
    return int(v.value)


def sb_set_cutoff(which: int, value: int, handle: Handle | None = None) -> None:
    """Set a small-problem cutoff on `handle` (default: the current device's)."""
    if handle is None:
        idx = torch.cuda.current_device()
        handle = _handles.get(idx) or _handles.setdefault(idx, Handle(idx))
    handle.check(load().sb_set_cutoff(handle.h, which, value))


def handle_for(t: torch.Tensor) -> Handle:
    idx = t.device.index if t.device.index is not None else torch.cuda.current_device()
    h = _handles.get(idx)
    if h is None:
        h = _handles[idx] = Handle(idx)
    return h


def sb_workspace_bytes(kind: int, dtype: int, layout: int, op: int, m: int, n: int,
                       handle: Handle | None = None) -> int:
    return int(load().sb_workspace_bytes(handle.h if handle else None, kind, dtype, layout, op, m, n))


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _dtype(t: torch.Tensor) -> int:
    if t.dtype not in _DTYPES:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return _DTYPES[t.dtype]


def _matrix_layout(M: torch.Tensor):
    """(layout, ld) of a 2-D tensor whose rows or columns are contiguous."""
    if M.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    r, c = M.shape
    sr, sc = M.stride()
    if M.numel() == 0:
        return SB_ROW_MAJOR, max(c, 1)
    if sc == 1 or c <= 1:
        return SB_ROW_MAJOR, (sr if r > 1 else max(c, 1))
    if sr == 1 or r <= 1:
        return SB_COL_MAJOR, (sc if c > 1 else max(r, 1))
    raise ValueError("matrix needs unit stride along rows or columns")


def _vec(v: torch.Tensor) -> torch.Tensor:
    if v.dim() != 1 or (v.numel() > 1 and v.stride(0) != 1):
        raise ValueError("vectors must be 1-D with unit stride")
    return v


def _device_check(*ts):
    d = ts[0].device
    for t in ts:
        if not t.is_cuda or t.device != d:
            raise ValueError("all operands must be on the same GPU")


def sb_gemv(A: torch.Tensor, x: torch.Tensor, c: torch.Tensor, op: int = SB_N) -> torch.Tensor:
    """c += op(A) x in place (row- or column-major A from its strides)."""
    _device_check(A, x, c)
    _vec(x), _vec(c)
    dt = _dtype(A)
    if x.dtype != A.dtype or c.dtype != A.dtype:
        raise TypeError("A, x and c must share a dtype")
    layout, ld = _matrix_layout(A)
    m, n = A.shape
    if x.numel() != (n if op == SB_N else m) or c.numel() != (m if op == SB_N else n):
        raise ValueError("x / c lengths do not match op(A)")
    h = handle_for(A)
    h.prepare(sb_workspace_bytes(SB_KIND_GEMV, dt, layout, op, m, n, h))
    h.check(load().sb_gemv(h.h, dt, layout, op, m, n, _ptr(A), ld, _ptr(x), _ptr(c)))
    return c


def sb_gemv_noalloc(A: torch.Tensor, x: torch.Tensor, c: torch.Tensor, op: int = SB_N) -> torch.Tensor:
    """c += op(A) x in place through the entry point that allocates nothing:
    the library's static per-GPU scratch replaces the workspace, and this
    wrapper allocates no device memory either (it only points the handle at
    the current stream)."""
    _device_check(A, x, c)
    _vec(x), _vec(c)
    dt = _dtype(A)
    if x.dtype != A.dtype or c.dtype != A.dtype:
        raise TypeError("A, x and c must share a dtype")
    layout, ld = _matrix_layout(A)
    m, n = A.shape
    if x.numel() != (n if op == SB_N else m) or c.numel() != (m if op == SB_N else n):
        raise ValueError("x / c lengths do not match op(A)")
    h = handle_for(A)
    h.prepare(0)
    h.check(load().sb_gemv_noalloc(h.h, dt, layout, op, m, n, _ptr(A), ld, _ptr(x), _ptr(c)))
    return c


def sb_gemv2(A: torch.Tensor, x: torch.Tensor, y: torch.Tensor, c: torch.Tensor, d: torch.Tensor):
    """c += A x and d += A^T y in place, reading A once (row- or column-major
    A from its strides)."""
    _device_check(A, x, y, c, d)
    _vec(x), _vec(y), _vec(c), _vec(d)
    dt = _dtype(A)
    if any(t.dtype != A.dtype for t in (x, y, c, d)):
        raise TypeError("A, x, y, c and d must share a dtype")
    layout, ld = _matrix_layout(A)
    m, n = A.shape
    if x.numel() != n or c.numel() != m or y.numel() != m or d.numel() != n:
        raise ValueError(f"A is {m}x{n}: need x, d of {n} and y, c of {m} entries")
    h = handle_for(A)
    h.prepare(sb_workspace_bytes(SB_KIND_GEMV2, dt, layout, 0, m, n, h))
    h.check(load().sb_gemv2(h.h, dt, layout, m, n, _ptr(A), ld, _ptr(x), _ptr(y), _ptr(c), _ptr(d)))
    return c, d


def sb_dot(x: torch.Tensor, y: torch.Tensor, alpha: torch.Tensor) -> torch.Tensor:
    """alpha (one-element device tensor) += x . y in place."""
    _device_check(x, y, alpha)
    _vec(x), _vec(y)
    dt = _dtype(x)
    if y.dtype != x.dtype or alpha.dtype != x.dtype or alpha.numel() != 1:
        raise TypeError("x, y and a one-element alpha must share a dtype")
    n = x.numel()
    if y.numel() != n:
        raise ValueError("x and y differ in length")
    h = handle_for(x)
    h.prepare(sb_workspace_bytes(SB_KIND_DOT, dt, 0, 0, 1, n, h))
    h.check(load().sb_dot(h.h, dt, n, _ptr(x), _ptr(y), _ptr(alpha)))
    return alpha


def sb_ger(x: torch.Tensor, y: torch.Tensor, C: torch.Tensor) -> torch.Tensor:
    """C += x (outer) y in place (row- or column-major C from its strides)."""
    _device_check(x, y, C)
    _vec(x), _vec(y)
    dt = _dtype(C)
    if x.dtype != C.dtype or y.dtype != C.dtype:
        raise TypeError("x, y and C must share a dtype")
    layout, ld = _matrix_layout(C)
    m, n = C.shape
    if x.numel() != m or y.numel() != n:
        raise ValueError("x must have C.shape[0] entries and y C.shape[1]")
    h = handle_for(C)
    h.prepare(0)
    h.check(load().sb_ger(h.h, dt, layout, m, n, _ptr(x), _ptr(y), _ptr(C), ld))
    return C


def _q_check(q: int, Aq: torch.Tensor):
    if q not in (SB_BF16, SB_FP8_E4M3):
        raise ValueError("q must be SB_BF16 or SB_FP8_E4M3")
    if Aq.element_size() != (2 if q == SB_BF16 else 1):
        raise TypeError("code tensor element size does not match q")


def sb_quantize_rows(A: torch.Tensor, Aq: torch.Tensor, scales: torch.Tensor, q: int):
    """Per-row scaled quantisation of a row-major binary32 A into Aq/scales."""
    _device_check(A, Aq, scales)
    _q_check(q, Aq)
    if A.dtype != torch.float32 or scales.dtype != torch.float32:
        raise TypeError("A and scales must be float32")
    la, lda = _matrix_layout(A)
    lq, ldq = _matrix_layout(Aq)
    if la != SB_ROW_MAJOR or lq != SB_ROW_MAJOR or A.shape != Aq.shape:
        raise ValueError("A and Aq must be row-major and of one shape")
    m, n = A.shape
    if scales.numel() != m:
        raise ValueError("scales must have one entry per row")
    h = handle_for(A)
    h.prepare(0)
    h.check(load().sb_quantize_rows(h.h, q, m, n, _ptr(A), lda, _ptr(Aq), ldq, _ptr(scales)))
    return Aq, scales


def sb_gemv_q(Aq: torch.Tensor, scales: torch.Tensor, x: torch.Tensor, c: torch.Tensor, q: int):
    """c += diag(scales) Q x in place, Q decoded from row-major codes Aq."""
    _device_check(Aq, scales, x, c)
    _q_check(q, Aq)
    _vec(x), _vec(c), _vec(scales)
    if x.dtype != torch.float32 or c.dtype != torch.float32 or scales.dtype != torch.float32:
        raise TypeError("scales, x and c must be float32")
    lq, ldq = _matrix_layout(Aq)
    if lq != SB_ROW_MAJOR:
        raise ValueError("Aq must be row-major")
    m, n = Aq.shape
    if x.numel() != n or c.numel() != m or scales.numel() != m:
        raise ValueError("x must have Aq.shape[1] entries, c and scales Aq.shape[0]")
    h = handle_for(Aq)
    h.prepare(sb_workspace_bytes(SB_KIND_GEMV_Q, q, 0, 0, m, n, h))
    h.check(load().sb_gemv_q(h.h, q, m, n, _ptr(Aq), ldq, _ptr(scales), _ptr(x), _ptr(c)))
    return c


def mx_row_bytes(q: int, n: int) -> int:
    """Bytes of element codes in one row of an MX matrix with n columns."""
    return n if q == SB_MXFP8_E4M3 else (n + 1) // 2


def mx_buffers(q: int, m: int, n: int, device=None):
    """Uninitialised (Q, S) device tensors for an m x n MX matrix: Q is
    m x ldq bytes with ldq the row's code bytes rounded up to 16, S is
    m x ceil(n/32) scale bytes."""
    if q not in (SB_MXFP8_E4M3, SB_MXFP4_E2M1):
        raise ValueError("q must be SB_MXFP8_E4M3 or SB_MXFP4_E2M1")
    ldq = max(16, (mx_row_bytes(q, n) + 15) // 16 * 16)
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    return (torch.empty((m, ldq), dtype=torch.uint8, device=dev),
            torch.empty((m, max(1, (n + 31) // 32)), dtype=torch.uint8, device=dev))


def _mx_check(Q: torch.Tensor, S: torch.Tensor, q: int, m: int, n: int):
    if Q.dtype != torch.uint8 or S.dtype != torch.uint8 or Q.dim() != 2 or S.dim() != 2:
        raise TypeError("Q and S must be 2-D uint8 tensors")
    if q not in (SB_MXFP8_E4M3, SB_MXFP4_E2M1):
        raise ValueError("q must be SB_MXFP8_E4M3 or SB_MXFP4_E2M1")
    if Q.shape[0] != m or S.shape[0] != m or Q.shape[1] < mx_row_bytes(q, n) or S.shape[1] < (n + 31) // 32:
        raise ValueError("Q or S too small for the matrix")
    if (m > 1 and (Q.stride(1) != 1 or S.stride(1) != 1)):
        raise ValueError("Q and S rows must be contiguous")


def sb_quantize_mx(A: torch.Tensor, Q: torch.Tensor, S: torch.Tensor, q: int):
    """MX quantisation of a row-major binary32 A into codes Q and scales S."""
    _device_check(A, Q, S)
    if A.dtype != torch.float32:
        raise TypeError("A must be float32")
    la, lda = _matrix_layout(A)
    if la != SB_ROW_MAJOR:
        raise ValueError("A must be row-major")
    m, n = A.shape
    _mx_check(Q, S, q, m, n)
    h = handle_for(A)
    h.prepare(0)
    h.check(load().sb_quantize_mx(h.h, q, m, n, _ptr(A), lda, _ptr(Q), Q.stride(0), _ptr(S), S.stride(0)))
    return Q, S


def sb_gemv_mx(Q: torch.Tensor, S: torch.Tensor, x: torch.Tensor, c: torch.Tensor, q: int) -> torch.Tensor:
    """c += (X * P) x in place for the MX matrix (Q, S) with x.numel() columns."""
    _device_check(Q, S, x, c)
    _vec(x), _vec(c)
    if x.dtype != torch.float32 or c.dtype != torch.float32:
        raise TypeError("x and c must be float32")
    m, n = c.numel(), x.numel()
    _mx_check(Q, S, q, m, n)
    h = handle_for(Q)
    h.prepare(sb_workspace_bytes(SB_KIND_GEMV_MX, q, 0, 0, m, n, h))
    h.check(load().sb_gemv_mx(h.h, q, m, n, _ptr(Q), Q.stride(0), _ptr(S), S.stride(0), _ptr(x), _ptr(c)))
    return c


def sb_dot2_f32(x: torch.Tensor, y: torch.Tensor, alpha: torch.Tensor) -> torch.Tensor:
    """Compensated binary32 alpha += x . y in place."""
    _device_check(x, y, alpha)
    _vec(x), _vec(y)
    if x.dtype != torch.float32 or y.dtype != torch.float32 or alpha.dtype != torch.float32:
        raise TypeError("sb_dot2_f32 takes float32 tensors")
    n = x.numel()
    if y.numel() != n or alpha.numel() != 1:
        raise ValueError("x and y differ in length or alpha is not one element")
    h = handle_for(x)
    h.prepare(sb_workspace_bytes(SB_KIND_DOT2, SB_F32, 0, 0, 1, n, h))
    h.check(load().sb_dot2_f32(h.h, n, _ptr(x), _ptr(y), _ptr(alpha)))
    return alpha


def sb_stream_read(src: torch.Tensor) -> None:
    """Measurement probe: stream the bytes of a contiguous device tensor."""
    if not src.is_cuda or not src.is_contiguous():
        raise ValueError("src must be a contiguous device tensor")
    nbytes = src.numel() * src.element_size()
    h = handle_for(src)
    h.prepare(sb_workspace_bytes(SB_KIND_PROBE_READ, 0, 0, 0, 0, nbytes, h))
    h.check(load().sb_stream_read(h.h, _ptr(src), nbytes))


def sb_stream_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    """Measurement probe: copy the bytes of src into dst (same byte size)."""
    _device_check(src, dst)
    if not src.is_contiguous() or not dst.is_contiguous():
        raise ValueError("src and dst must be contiguous")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    h = handle_for(src)
    h.prepare(0)
    h.check(load().sb_stream_copy(h.h, _ptr(src), _ptr(dst), nbytes))


def sb_stream_update(C: torch.Tensor) -> None:
    """Measurement probe: read and rewrite a row-major float64 matrix in
    place with GER's access pattern (its value does not change)."""
    if not C.is_cuda or C.dtype != torch.float64 or C.dim() != 2:
        raise ValueError("C must be a 2-D float64 device tensor")
    layout, ld = _matrix_layout(C)
    if layout != SB_ROW_MAJOR:
        raise ValueError("C must be row-major")
    h = handle_for(C)
    h.prepare(0)
    h.check(load().sb_stream_update(h.h, _ptr(C), C.shape[0], C.shape[1], ld))


class GemvProblem:
    """One problem c += op(A) x (or c += diag(scales) Q x for codes).

    A is a 2-D device tensor with unit stride along its rows or its columns
    (float64/float32 with op SB_N or SB_T; or row-major 2-byte / 1-byte codes
    with q = SB_BF16 / SB_FP8_E4M3, scales and op SB_N); group /
    rows_per_tile / split select the launch configuration (0: automatic).
    """

    __slots__ = ("A", "x", "c", "scales", "q", "group", "rows_per_tile", "split", "op")

    def __init__(self, A, x, c, scales=None, q=None, group=0, rows_per_tile=0, split=0, op=SB_N):
        self.A, self.x, self.c, self.scales, self.q = A, x, c, scales, q
        self.group, self.rows_per_tile, self.split = group, rows_per_tile, split
        self.op = op

    def dtype(self) -> int:
        if self.q is not None:
            return self.q
        return _dtype(self.A)


def make_descs(problems) -> "ctypes.Array":
    """Marshal a list of GemvProblem into a C array of sb_gemv_desc."""
    arr = (sb_gemv_desc * max(len(problems), 1))()
    for i, p in enumerate(problems):
        layout, ld = _matrix_layout(p.A)
        m, n = p.A.shape
        dt = p.dtype()
        if p.op not in (SB_N, SB_T):
            raise ValueError("op must be SB_N or SB_T")
        if dt in (SB_BF16, SB_FP8_E4M3):
            if layout != SB_ROW_MAJOR or p.op != SB_N:
                raise ValueError("quantised batched problems are row-major N (the scales belong to rows)")
            _q_check(dt, p.A)
            if p.scales is None or p.scales.numel() != m or p.x.dtype != torch.float32 or p.c.dtype != torch.float32:
                raise ValueError("quantised problems need m scales and float32 x, c")
        elif p.x.dtype != p.A.dtype or p.c.dtype != p.A.dtype:
            raise TypeError("A, x and c must share a dtype")
        _vec(p.x), _vec(p.c)
        xl, cl = (n, m) if p.op == SB_N else (m, n)
        if p.x.numel() != xl or p.c.numel() != cl:
            raise ValueError("x must have n entries and c m (op N), or x m and c n (op T)")
        d = arr[i]
        d.dtype, d.group, d.rows_per_tile, d.split = dt, p.group, p.rows_per_tile, p.split
        d.m, d.n, d.lda = m, n, ld
        d.layout, d.op = layout, p.op
        d.A, d.x, d.c = p.A.data_ptr(), p.x.data_ptr(), p.c.data_ptr()
        d.scales = p.scales.data_ptr() if p.scales is not None else None
    return arr


def sb_gemv_batched_table_bytes(problems) -> tuple[int, int]:
    descs = make_descs(problems)
    img = ctypes.c_size_t(0)
    total = load().sb_gemv_batched_table_bytes(descs, len(problems), ctypes.byref(img))
    if total == (1 << 64) - 1:
        raise StreamBlasError(SB_EINVAL, "invalid batched descriptors")
    return int(total), int(img.value)


def sb_gemv_batched_resolve(problems) -> list[dict]:
    """The (group, rows_per_tile, split) the batched kernel will use per problem."""
    descs = make_descs(problems)
    out = (sb_gemv_desc * max(len(problems), 1))()
    st = load().sb_gemv_batched_resolve(descs, len(problems), out)
    if st != SB_OK:
        raise StreamBlasError(st, load().sb_last_error(None).decode())
    return [{"group": out[i].group, "rows_per_tile": out[i].rows_per_tile, "split": out[i].split}
            for i in range(len(problems))]


def sb_gemv_batched(problems) -> None:
    """All problems in one persistent launch on the current stream."""
    if not problems:
        return
    descs = make_descs(problems)
    total, _ = sb_gemv_batched_table_bytes(problems)
    h = handle_for(problems[0].A)
    h.prepare(total)
    h.check(load().sb_gemv_batched(h.h, descs, len(problems)))


class Plan:
    """A batched plan (sb_plan_*): the problems are encoded once into the
    workspace of a handle private to the plan, and run() launches them on
    the current stream with no host work (a captured run() can be replayed).
    The plan keeps the problems' tensors alive."""

    def __init__(self, problems, device=None):
        self.problems = list(problems)
        dev = self.problems[0].A.device if self.problems else device
        self.handle = Handle(dev)
        total, _ = sb_gemv_batched_table_bytes(self.problems) if self.problems else (0, 0)
        self.handle.prepare(total)
        self._descs = make_descs(self.problems) if self.problems else (sb_gemv_desc * 1)()
        p = ctypes.c_void_p()
        self.handle.check(load().sb_plan_create(self.handle.h, self._descs, len(self.problems), ctypes.byref(p)))
        self.p = p

    def run(self) -> None:
        self.handle.prepare(0)  # the current stream
        self.handle.check(load().sb_plan_run(self.p))

    def __del__(self):
        if getattr(self, "p", None) and _lib is not None:
            _lib.sb_plan_destroy(self.p)
            self.p = None


class BatchTable:
    """A device batch table at a fixed address plus a pinned host image.

    encode() writes the table for a list of problems into the pinned image and
    copies it to the device table on the current stream; run() launches the
    persistent kernel over it.  Because the kernel reads the tile count from
    the table, a run() captured in a HIP graph can be replayed after encode()
    has written a new batch to the same address.
    """

    def __init__(self, capacity_bytes: int, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.capacity = int(capacity_bytes)
        self.dev = torch.empty(self.capacity, dtype=torch.uint8, device=self.device)
        self.host = torch.empty(self.capacity, dtype=torch.uint8, pin_memory=True)
        self.h = Handle(self.device.index)
        self._copied = None  # event after the last host-to-device copy of the image

    def fits(self, problems) -> bool:
        return sb_gemv_batched_table_bytes(problems)[0] <= self.capacity

    def encode(self, problems) -> None:
        self.encode_descs(make_descs(problems), len(problems))

    def encode_descs(self, descs, count: int) -> None:
        """Encode `count` sb_gemv_desc structs at `descs` (a ctypes array or
        a pointer to structs laid out like sb_gemv_desc)."""
        if not isinstance(descs, ctypes.Array):
            descs = ctypes.cast(descs, ctypes.POINTER(sb_gemv_desc))
        img_c = ctypes.c_size_t(0)
        total = load().sb_gemv_batched_table_bytes(descs, count, ctypes.byref(img_c))
        if total == (1 << 64) - 1:
            raise StreamBlasError(SB_EINVAL, "invalid batched descriptors")
        img = int(img_c.value)
        if total > self.capacity:
            raise StreamBlasError(SB_ENOMEM, f"batch table needs {total} bytes, capacity {self.capacity}")
        if self._copied is not None:
            self._copied.synchronize()  # the pinned image may still be in flight
        st = load().sb_gemv_batched_encode(descs, count, ctypes.c_void_p(self.dev.data_ptr()),
                                           ctypes.c_void_p(self.host.data_ptr()), img)
        if st != SB_OK:
            raise StreamBlasError(st, load().sb_last_error(None).decode())
        self.dev[:img].copy_(self.host[:img], non_blocking=True)
        self._copied = torch.cuda.Event()
        self._copied.record()

    def run(self, grid: int = 0) -> None:
        self.h.prepare(0)
        self.h.check(load().sb_gemv_batched_run(self.h.h, ctypes.c_void_p(self.dev.data_ptr()), grid))


def sb_fill_uniform(out: torch.Tensor, seed: int, counter0: int = 0) -> torch.Tensor:
    """Fill a contiguous float64/float32 device tensor with SplitMix64 uniforms in [-1, 1)."""
    if not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous device tensor")
    dt = _dtype(out)
    h = handle_for(out)
    h.prepare(0)
    h.check(load().sb_fill_uniform(h.h, dt, _ptr(out), out.numel(), seed & ((1 << 64) - 1), counter0))
    return out
