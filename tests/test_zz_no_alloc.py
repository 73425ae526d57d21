"""sb_gemv_noalloc, the GEMV entry point that allocates nothing: through the
C-ABI its results equal sb_gemv's bit for bit (same kernels, same order;
only the home of the split partial sums differs) and lie within the GEMV
bound of the CPU oracle, on calls in a row whose shapes shrink, so a later
call finds the previous call's partial sums in the shared static scratch."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import U32, U64, assert_within, dev, gemv_bound, host

pytestmark = pytest.mark.gpu


def gemv_both(sb, A, x, c0, op):
    """(sb_gemv result, sb_gemv_noalloc result) on copies of c0."""
    Ad, xd = dev(A), dev(x)
    c_ws, c_na = dev(c0), dev(c0)
    sb.sb_gemv(Ad, xd, c_ws, op=op)
    sb.sb_gemv_noalloc(Ad, xd, c_na, op=op)
    return host(c_ws), host(c_na)


# Each sequence: shapes that need split partial sums (column splits for
# kernel N on short-wide rows, row splits for kernel T), largest first.
SEQUENCES = [
    ("f64 T", np.float64, 1, [(65536, 4096), (1024, 1024)]),
    ("f64 N", np.float64, 0, [(256, 262144), (1024, 16384)]),
    ("f32 T", np.float32, 1, [(16384, 8192), (300, 5000)]),
    ("f32 N", np.float32, 0, [(8, 1 << 22), (64, 70001)]),
]


@pytest.mark.parametrize("name,npd,op,shapes", SEQUENCES, ids=[s[0] for s in SEQUENCES])
def test_noalloc_matches_gemv_on_shrinking_calls(sb, name, npd, op, shapes):
    dt = 0 if npd == np.float64 else 1
    for k, (m, n) in enumerate(shapes):
        need = sb.sb_workspace_bytes(sb.SB_KIND_GEMV, dt, 0, op, m, n)
        assert 0 < need <= 4 << 20, (m, n, need)
        A, x, c0 = workloads.gemv_inputs(m, n, seed=900 + k, dist="normal", op_t=bool(op), dtype=npd)
        print(f"{name} {m}x{n}: {need} bytes of partial sums", flush=True)
        got_ws, got_na = gemv_both(sb, A, x, c0, op)
        assert np.array_equal(got_ws.view(np.uint8), got_na.view(np.uint8)), (name, m, n)
        ref = oracle.gemv(A, x, c0, op=op)
        K = n if op == 0 else m
        assert_within(got_na, ref, gemv_bound(A, x, c0, op, K, U64 if npd == np.float64 else U32),
                      f"noalloc {name} {m}x{n}")


def test_noalloc_integer_exact_and_unsplit(sb):
    """Integer data: bit-exact against the oracle; a shape with no split
    (no scratch) and one with a split, in a row."""
    for (m, n, op) in ((1024, 1024, 0), (2048, 2048, 1)):
        A, x, c0 = workloads.gemv_inputs(m, n, seed=77, dist="int8", op_t=bool(op))
        got_ws, got_na = gemv_both(sb, A, x, c0, op)
        assert np.array_equal(got_na, oracle.gemv(A, x, c0, op=op))
        assert np.array_equal(got_ws, got_na)


def test_noalloc_through_c_abi_rejects_oversized_and_keeps_workspace(sb):
    """Direct C-ABI calls on a handle with no workspace: the oversized shape
    returns SB_ENOMEM (its partial sums would need 32 MiB), a fitting split
    shape runs, and sb_gemv on the same workspace-less handle refuses it."""
    L = sb.load()
    h = ctypes.c_void_p()
    stream = torch.cuda.current_stream().cuda_stream
    assert L.sb_handle_create(None, 0, ctypes.c_void_p(stream), ctypes.byref(h)) == 0
    try:
        fake_a, fake_x, fake_c = 1 << 44, 1 << 45, (1 << 45) + (1 << 40)
        st = L.sb_gemv_noalloc(h, 0, 0, 0, 65536, 262144, fake_a, 262144, fake_x, fake_c)
        assert st == sb.SB_ENOMEM and b"static scratch" in L.sb_last_error(h)
        m, n = 256, 262144
        A, x, c0 = workloads.gemv_inputs(m, n, seed=5, dist="int8")
        Ad, xd, cd = dev(A), dev(x), dev(c0)
        assert L.sb_gemv(h, 0, 0, 0, m, n, Ad.data_ptr(), n, xd.data_ptr(), cd.data_ptr()) == sb.SB_ENOMEM
        assert L.sb_gemv_noalloc(h, 0, 0, 0, m, n, Ad.data_ptr(), n, xd.data_ptr(), cd.data_ptr()) == 0
        assert np.array_equal(host(cd), oracle.gemv(A, x, c0))
    finally:
        L.sb_handle_destroy(h)
