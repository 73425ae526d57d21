"""The C-ABI on the CPU: the library loads, exports every function the
header declares, and rejects invalid calls before any device work (so these
calls are safe without a GPU; the pointers below are never dereferenced)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "streamblas.h")


@pytest.fixture(scope="module")
def L():
    import paper_2108_02025_amd as sb
    if not os.path.exists(sb.lib_path):
        from paper_2108_02025_amd import build
        build.build(verbose=False)
    return sb.load()


@pytest.fixture()
def h(L):
    hd = ctypes.c_void_p()
    assert L.sb_handle_create(None, 0, None, ctypes.byref(hd)) == 0
    yield hd
    L.sb_handle_destroy(hd)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sb_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name


def test_version_and_status_strings(L):
    assert L.sb_version() == 100
    assert L.sb_status_string(0) == b"success"
    assert L.sb_status_string(-1) == b"invalid argument"
    assert L.sb_status_string(-2) == b"workspace too small"
    assert L.sb_status_string(-4) == b"unsupported combination"
    assert L.sb_status_string(7) == b"unknown status"


FAKE = 1 << 40          # 16-byte aligned fake device addresses, never touched
A_, X_, C_ = FAKE, FAKE + (1 << 36), FAKE + (2 << 36)


def gemv(L, h, dt=0, layout=0, op=0, m=10, n=10, A=A_, lda=10, x=X_, c=C_):
    return L.sb_gemv(h, dt, layout, op, m, n, A, lda, x, c)


def test_gemv_validation(L, h):
    assert gemv(L, None) == -1
    assert gemv(L, h, dt=2) == -4 and gemv(L, h, dt=3) == -4
    assert gemv(L, h, dt=9) == -1
    assert gemv(L, h, layout=2) == -1 and gemv(L, h, op=5) == -1
    assert gemv(L, h, m=-1) == -1 and gemv(L, h, n=-3) == -1
    assert gemv(L, h, lda=9) == -1                      # row-major needs lda >= n
    assert gemv(L, h, layout=1, m=12, n=5, lda=11) == -1  # column-major needs lda >= m
    assert b"lda" in L.sb_last_error(h)
    assert gemv(L, h, A=None) == -1 and gemv(L, h, x=None) == -1 and gemv(L, h, c=None) == -1
    assert gemv(L, h, A=A_ + 4) == -1                   # not 8-byte aligned for binary64
    assert gemv(L, h, c=A_ + 80) == -1                  # c inside A
    assert gemv(L, h, c=X_ + 8) == -1                   # c overlaps x
    assert gemv(L, h, m=1 << 40, n=1 << 40, lda=1 << 40) == -1  # extent overflow
    # empty outputs / reductions return before any launch, null pointers allowed
    assert gemv(L, h, m=0, A=None, x=None, c=None) == 0
    assert gemv(L, h, n=0, lda=1, A=None, x=None) == 0
    assert gemv(L, h, op=1, m=0, c=None, A=None, x=None) == 0


def test_workspace_sizing_and_enomem(L, h):
    ws = L.sb_workspace_bytes
    assert ws(None, 0, 0, 0, 0, 1024, 1024) == 0          # x fits in LDS: no split
    short_wide = ws(None, 0, 0, 0, 0, 256, 262144)
    assert short_wide > 0 and short_wide % (256 * 8) == 0
    assert ws(None, 0, 0, 1, 1, 262144, 256) == short_wide  # column-major T: same kernel and plan
    assert ws(None, 0, 2, 0, 0, 5, 5) == (1 << 64) - 1      # narrow dtype is not a plain GEMV
    assert ws(None, 1, 0, 0, 0, 1, 1 << 28) > 0            # DOT partial sums
    assert ws(None, 2, 0, 0, 0, 100, 100) == 0             # GER needs none
    assert ws(None, 4, 1, 0, 0, 1, 1 << 27) == 2 * ws(None, 1, 1, 0, 0, 1, 1 << 27)
    # no workspace on the handle: calls that need it fail before launching
    assert gemv(L, h, m=256, n=262144, lda=262144, x=X_, c=C_) == -2
    assert b"workspace" in L.sb_last_error(h)
    assert L.sb_dot(h, 0, 1 << 20, X_, A_, C_) == -2
    assert L.sb_dot2_f32(h, 1 << 20, X_, A_, C_) == -2


def test_dot_ger_quant_validation(L, h):
    assert L.sb_dot(h, 0, -1, X_, A_, C_) == -1
    assert L.sb_dot(h, 0, 10, X_, A_, None) == -1
    assert L.sb_dot(h, 0, 10, X_, A_, X_ + 16) == -1       # alpha inside x
    assert L.sb_dot(h, 2, 10, X_, A_, C_) == -4
    assert L.sb_dot(h, 0, 0, None, None, C_) == 0           # empty: alpha unchanged, no launch
    assert L.sb_ger(h, 0, 0, 4, 5, X_, A_, C_, 4) == -1     # ldc < n
    assert L.sb_ger(h, 0, 0, 4, 5, C_ + 8, A_, C_, 5) == -1  # x inside C
    assert L.sb_ger(h, 0, 0, 0, 5, None, None, None, 5) == 0
    assert L.sb_quantize_rows(h, 0, 4, 4, A_, 4, C_, 4, X_) == -1   # q must be narrow
    assert L.sb_quantize_rows(h, 2, 4, 4, A_, 3, C_, 4, X_) == -1   # lda < n
    assert L.sb_quantize_rows(h, 2, 4, 4, A_, 4, A_, 4, X_) == -1   # Aq overlaps A
    assert L.sb_gemv_q(h, 1, 4, 4, A_, 4, X_, X_, C_) == -1          # q must be narrow
    assert L.sb_gemv_q(h, 3, 4, 4, A_, 4, X_, X_ + 64, X_ + 4) == -1  # c overlaps scales
    assert L.sb_dot2_f32(h, 5, X_ + 2, A_, C_) == -1                 # misaligned x


def test_handle_errors(L):
    assert L.sb_handle_create(None, 16, None, None) == -1
    hd = ctypes.c_void_p()
    assert L.sb_handle_create(None, 16, None, ctypes.byref(hd)) == -1
    assert b"workspace" in L.sb_last_error(None)
    assert L.sb_set_stream(None, None) == -1
    assert L.sb_handle_destroy(None) == 0
