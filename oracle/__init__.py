"""CPU oracle for the streaming BLAS-1/2 operations of Singh and Bassoy,
"High Performance Level-1 and Level-2 BLAS" (arXiv 2108.02025).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow statement of what
the GPU library computes.  Only the test suite, the package smoke check and
the CPU-baseline leg of ``bench.py`` may import it; the GPU library never
does, and the two share no code.

Everything is evaluated by ``oracle.c`` (built with gcc -O2
-ffp-contract=off): binary64, products rounded on their own, sums in
ascending index order from +0.0, initial output added last (section 3.1
problem definitions).  This module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ROW_MAJOR, COL_MAJOR = 0, 1
OP_N, OP_T = 0, 1
Q_BF16, Q_E4M3 = 2, 3
Q_MXFP8, Q_MXFP4 = 4, 5

_CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared", "-Wall"]


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64, I32, D, F = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_float
        L.orc_gemv.argtypes = [I32, I32, I64, I64, P, I64, P, P]
        L.orc_gemv.restype = I32
        L.orc_gemv_entries.argtypes = [I32, I32, I64, I64, P, I64, P, P, I64, P, P]
        L.orc_gemv_entries.restype = I32
        L.orc_dot.argtypes = [I64, P, P, D]
        L.orc_dot.restype = D
        L.orc_ger.argtypes = [I32, I64, I64, P, P, P, I64]
        L.orc_ger.restype = I32
        L.orc_bf16_from_f32.argtypes = [F]
        L.orc_bf16_from_f32.restype = ctypes.c_uint16
        L.orc_bf16_to_f32.argtypes = [ctypes.c_uint16]
        L.orc_bf16_to_f32.restype = F
        L.orc_e4m3_from_f32.argtypes = [F]
        L.orc_e4m3_from_f32.restype = ctypes.c_uint8
        L.orc_e4m3_to_f32.argtypes = [ctypes.c_uint8]
        L.orc_e4m3_to_f32.restype = F
        L.orc_quantize_rows.argtypes = [I32, I64, I64, P, I64, P, I64, P]
        L.orc_quantize_rows.restype = I32
        L.orc_gemv_q.argtypes = [I32, I64, I64, P, I64, P, P, P]
        L.orc_gemv_q.restype = I32
        L.orc_dot_exact_f32.argtypes = [I64, P, P, F, I32]
        L.orc_dot_exact_f32.restype = D
        L.orc_e8m0_to_f64.argtypes = [ctypes.c_uint8]
        L.orc_e8m0_to_f64.restype = D
        L.orc_e2m1_to_f64.argtypes = [ctypes.c_uint8]
        L.orc_e2m1_to_f64.restype = D
        L.orc_e2m1_from_f64.argtypes = [D]
        L.orc_e2m1_from_f64.restype = ctypes.c_uint8
        L.orc_quantize_mx.argtypes = [I32, I64, I64, P, I64, P, I64, P, I64]
        L.orc_quantize_mx.restype = I32
        L.orc_gemv_mx.argtypes = [I32, I64, I64, P, I64, P, I64, P, P]
        L.orc_gemv_mx.restype = I32
        L.orc_sum_exact_f64.argtypes = [I64, P]
        L.orc_sum_exact_f64.restype = D
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _storage(A: np.ndarray, layout: int):
    """Return (flat binary64 buffer, lda) of a 2-D array in the given layout."""
    A = np.asarray(A, dtype=np.float64)
    if layout == ROW_MAJOR:
        A = np.ascontiguousarray(A)
        return A.reshape(-1), max(A.shape[1], 1)
    A = np.asfortranarray(A)
    return A.reshape(-1, order="F"), max(A.shape[0], 1)


def gemv(A, x, c0, op: int = OP_N, layout: int = ROW_MAJOR, lda: int | None = None,
         shape: tuple[int, int] | None = None) -> np.ndarray:
    """c0 + op(A) x per the GEMV definition (section 3.1).

    ``A`` is either a 2-D array (stored here in ``layout``) or, with
    ``shape=(m, n)`` and ``lda``, a flat buffer already in that layout.
    Returns a new binary64 vector.
    """
    if shape is None:
        m, n = np.shape(A)
        buf, ld = _storage(A, layout)
    else:
        m, n = shape
        buf, ld = _f64(A).reshape(-1), lda
    x = _f64(x)
    c = _f64(c0).copy()
    assert x.shape[0] == (n if op == OP_N else m)
    assert c.shape[0] == (m if op == OP_N else n)
    rc = lib().orc_gemv(layout, op, m, n, _p(buf), ld, _p(x), _p(c))
    assert rc == 0, rc
    return c


def gemv2(A, x, y, c0, d0, layout: int = ROW_MAJOR) -> tuple[np.ndarray, np.ndarray]:
    """Two-sided GEMV: (c0 + A x, d0 + A^T y), each by the GEMV definition
    (section 3.1) on its own; the fused form reads A once but computes the
    same two sums."""
    return gemv(A, x, c0, op=OP_N, layout=layout), gemv(A, y, d0, op=OP_T, layout=layout)


def gemv_entries(A, x, idx, c0_at_idx, op: int = OP_N, layout: int = ROW_MAJOR,
                 lda: int | None = None, shape: tuple[int, int] | None = None) -> np.ndarray:
    """The GEMV definition evaluated only for the output indices ``idx``."""
    if shape is None:
        m, n = np.shape(A)
        buf, ld = _storage(A, layout)
    else:
        m, n = shape
        buf, ld = _f64(A).reshape(-1), lda
    x = _f64(x)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    c0 = _f64(c0_at_idx)
    out = np.empty(idx.shape[0], dtype=np.float64)
    rc = lib().orc_gemv_entries(layout, op, m, n, _p(buf), ld, _p(x), _p(idx), idx.shape[0],
                                _p(c0), _p(out))
    assert rc == 0, rc
    return out


def dot(x, y, alpha0: float = 0.0) -> float:
    """alpha0 + x . y per the DOT definition (section 3.1)."""
    x, y = _f64(x), _f64(y)
    assert x.shape == y.shape
    return float(lib().orc_dot(x.shape[0], _p(x), _p(y), float(alpha0)))


def ger(x, y, C0, layout: int = ROW_MAJOR) -> np.ndarray:
    """C0 + x (outer) y per the GEM definition (section 3.1); returns a new 2-D array."""
    x, y = _f64(x), _f64(y)
    m, n = x.shape[0], y.shape[0]
    buf, ld = _storage(C0, layout)
    buf = buf.copy()
    rc = lib().orc_ger(layout, m, n, _p(x), _p(y), _p(buf), ld)
    assert rc == 0, rc
    if layout == ROW_MAJOR:
        return buf.reshape(m, n)
    return buf.reshape(n, m).T


def bf16_from_f32(v: float) -> int:
    return int(lib().orc_bf16_from_f32(float(v)))


def bf16_to_f32(code: int) -> float:
    return float(lib().orc_bf16_to_f32(int(code)))


def e4m3_from_f32(v: float) -> int:
    return int(lib().orc_e4m3_from_f32(float(v)))


def e4m3_to_f32(code: int) -> float:
    return float(lib().orc_e4m3_to_f32(int(code)))


def quantize_rows(A, q: int):
    """Per-row scaled quantisation of a binary32 matrix; returns (codes, scales)."""
    A = np.ascontiguousarray(A, dtype=np.float32)
    m, n = A.shape
    codes = np.zeros((m, n), dtype=np.uint16 if q == Q_BF16 else np.uint8)
    scales = np.zeros(m, dtype=np.float32)
    rc = lib().orc_quantize_rows(q, m, n, _p(A), max(n, 1), _p(codes), max(n, 1), _p(scales))
    assert rc == 0, rc
    return codes, scales


def gemv_q(codes, scales, x, c0, q: int) -> np.ndarray:
    """c0 + diag(s) Q x in binary64 on the decoded codes."""
    codes = np.ascontiguousarray(codes)
    m, n = codes.shape
    scales = np.ascontiguousarray(scales, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32)
    c = _f64(c0).copy()
    rc = lib().orc_gemv_q(q, m, n, _p(codes), max(n, 1), _p(scales), _p(x), _p(c))
    assert rc == 0, rc
    return c


def e8m0_to_f64(code: int) -> float:
    return float(lib().orc_e8m0_to_f64(int(code)))


def e2m1_to_f64(code: int) -> float:
    return float(lib().orc_e2m1_to_f64(int(code)))


def e2m1_from_f64(v: float) -> int:
    return int(lib().orc_e2m1_from_f64(float(v)))


def mx_row_bytes(q: int, n: int) -> int:
    """Bytes of one row of MX element codes (MXFP8: n, MXFP4: ceil(n/2))."""
    return n if q == Q_MXFP8 else (n + 1) // 2


def quantize_mx(A, q: int):
    """MX quantisation (blocks of 32 along each row) of a binary32 matrix;
    returns (codes m x row bytes, E8M0 scales m x ceil(n/32))."""
    A = np.ascontiguousarray(A, dtype=np.float32)
    m, n = A.shape
    rb, nb = mx_row_bytes(q, n), (n + 31) // 32
    codes = np.zeros((m, max(rb, 1)), dtype=np.uint8)
    scales = np.zeros((m, max(nb, 1)), dtype=np.uint8)
    rc = lib().orc_quantize_mx(q, m, n, _p(A), max(n, 1), _p(codes), codes.shape[1], _p(scales), scales.shape[1])
    assert rc == 0, rc
    return codes[:, :rb], scales[:, :nb]


def gemv_mx(codes, scales, x, c0, q: int, n: int) -> np.ndarray:
    """c0 + (X * P) x in binary64 on the decoded MX blocks of an m x n matrix."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    scales = np.ascontiguousarray(scales, dtype=np.uint8)
    m = codes.shape[0]
    x = np.ascontiguousarray(x, dtype=np.float32)
    assert x.shape[0] == n
    c = _f64(c0).copy()
    rc = lib().orc_gemv_mx(q, m, n, _p(codes), max(codes.shape[1], 1), _p(scales), max(scales.shape[1], 1),
                           _p(x), _p(c))
    assert rc == 0, rc
    return c


def dot_exact_f32(x, y, alpha0: float = 0.0, absval: bool = False) -> float:
    """Exact alpha0 + x . y of binary32 inputs, rounded once to binary64."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    assert x.shape == y.shape
    return float(lib().orc_dot_exact_f32(x.shape[0], _p(x), _p(y), float(alpha0), int(absval)))


def sum_exact_f64(v) -> float:
    v = _f64(v)
    return float(lib().orc_sum_exact_f64(v.shape[0], _p(v)))
