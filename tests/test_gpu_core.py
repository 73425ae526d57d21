"""GPU parity of GEMV, DOT and GER against the CPU oracle at sizes the
oracle finishes in seconds: several tiles, ragged tails, edge sizes, every
(layout, op) pair, padded leading dimensions, misaligned bases, special
values and repeat-run determinism.  Every call goes through the C-ABI."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import U32, U64, assert_within, dev, gemv_bound, host, normwise

pytestmark = pytest.mark.gpu

NP = {0: np.float64, 1: np.float32}
TT = {np.float64: torch.float64, np.float32: torch.float32}


def as_layout(A, layout):
    """Device tensor of logical shape A.shape stored row- or column-major."""
    if layout == 0:
        return dev(A)
    return dev(np.ascontiguousarray(A.T)).t()


def run_gemv(sb, A, x, c0, op, layout):
    Ad = as_layout(A, layout)
    xd, cd = dev(x), dev(c0)
    sb.sb_gemv(Ad, xd, cd, op=op)
    return host(cd)


# ------------------------------------------------------------------ GEMV ----

@pytest.mark.parametrize("op", [0, 1])
@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("cdist", ["int8", "uniform"])
def test_gemv_1024_integer_bit_exact(sb, op, layout, cdist):
    """1024x1024 with A, x in [-8, 8] integers: every partial sum is exact,
    so any correct order gives the oracle's bits (also with c0 uniform: the
    exact sum plus c0 is a single rounding)."""
    A, x, c0 = workloads.gemv_inputs(1024, 1024, seed=102, dist="int8", op_t=bool(op), c_dist=cdist)
    ref = oracle.gemv(A, x, c0, op=op, layout=layout)
    got = run_gemv(sb, A, x, c0, op, layout)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("op", [0, 1])
@pytest.mark.parametrize("layout", [0, 1])
def test_gemv_1024_uniform_bound(sb, op, layout):
    A, x, c0 = workloads.gemv_inputs(1024, 1024, seed=101, op_t=bool(op))
    ref = oracle.gemv(A, x, c0, op=op)
    got = run_gemv(sb, A, x, c0, op, layout)
    assert_within(got, ref, gemv_bound(A, x, c0, op, 1024, U64), "gemv 1024")


@pytest.mark.parametrize("dt", [0, 1])
@pytest.mark.parametrize("op", [0, 1])
@pytest.mark.parametrize("m,n", [(1, 1), (1, 7), (7, 1), (2, 3), (3, 2), (63, 65), (64, 64), (65, 63),
                                 (127, 129), (129, 4093), (4093, 129), (5, 33000), (33000, 5),
                                 (300, 40000), (17, 70001),
                                 # launch-shape boundaries: x just above 40 KiB, 80 KiB, 128 KiB
                                 (37, 10241), (21, 20483), (13, 16384), (11, 16387)])
def test_gemv_edge_sizes(sb, dt, op, m, n):
    npd = NP[dt]
    A, x, c0 = workloads.gemv_inputs(m, n, seed=m * 7 + n, dist="normal", op_t=bool(op), dtype=npd)
    ref = oracle.gemv(A, x, c0, op=op)
    K = n if op == 0 else m
    for layout in (0, 1):
        got = run_gemv(sb, A, x, c0, op, layout)
        assert_within(got, ref, gemv_bound(A, x, c0, op, K, U64 if dt == 0 else U32), f"{m}x{n}")
        if dt == 1:
            assert normwise(got, ref) < 2.0 ** -16
    # integer data is bit-exact whatever the tiling
    Ai, xi, ci = workloads.gemv_inputs(m, n, seed=3, dist="int7" if dt else "int8", op_t=bool(op), dtype=npd)
    if dt == 0 or K <= 1 << 16:
        assert np.array_equal(run_gemv(sb, Ai, xi, ci, op, 0), oracle.gemv(Ai, xi, ci, op=op))


@pytest.mark.parametrize("dt", [0, 1])
@pytest.mark.parametrize("m,n", [(512, 16384), (1024, 16384), (1000, 20001), (2048, 16384)])
def test_gemv_few_long_rows_split(sb, dt, m, n):
    """Few rows of a large operand: the row-dot plan splits the columns so
    that every compute unit has waves (partial sums, then the ordered second
    stage).  Row-major N and column-major T take that path."""
    npd = NP[dt]
    assert sb.sb_workspace_bytes(sb.SB_KIND_GEMV, dt, 0, 0, m, n) > 0, "expected a column split"
    A, x, c0 = workloads.gemv_inputs(m, n, seed=m + n, dist="normal", dtype=npd)
    ref = oracle.gemv(A, x, c0)
    got = run_gemv(sb, A, x, c0, 0, 0)
    assert_within(got, ref, gemv_bound(A, x, c0, 0, n, U64 if dt == 0 else U32), f"{m}x{n}")
    got_t = run_gemv(sb, np.ascontiguousarray(A.T), x, c0, 1, 1)  # column-major T of A^T
    assert np.array_equal(got_t, got)
    Ai, xi, ci = workloads.gemv_inputs(m, n, seed=5, dist="int7" if dt else "int8", dtype=npd)
    assert np.array_equal(run_gemv(sb, Ai, xi, ci, 0, 0), oracle.gemv(Ai, xi, ci))


@pytest.mark.parametrize("dt", [0, 1])
def test_gemv_layout_equivalence_bitwise(sb, dt):
    """(row-major, N) and (column-major, T) on one buffer are the same
    computation; so are (row-major, T) and (column-major, N)."""
    npd = NP[dt]
    m, n = 777, 1531
    A, x, c0 = workloads.gemv_inputs(m, n, seed=5, dist="normal", dtype=npd)
    buf = dev(A)                         # m x n row-major == n x m column-major
    colview = buf.reshape(-1).as_strided((n, m), (1, n))
    c1, c2 = dev(c0), dev(c0)
    sb.sb_gemv(buf, dev(x), c1, op=0)
    sb.sb_gemv(colview, dev(x), c2, op=1)
    assert torch.equal(c1, c2)
    xt = dev(workloads.gemv_inputs(m, 1, seed=6, dtype=npd)[0].reshape(-1))
    ct = dev(np.zeros(n, npd))
    d1, d2 = ct.clone(), ct.clone()
    sb.sb_gemv(buf, xt, d1, op=1)
    sb.sb_gemv(colview, xt, d2, op=0)
    assert torch.equal(d1, d2)


@pytest.mark.parametrize("dt", [0, 1])
@pytest.mark.parametrize("op", [0, 1])
def test_gemv_padded_lda_and_misaligned_base(sb, dt, op):
    """lda > n (padding holds NaN, so any read of it would poison the
    result) and a base pointer one element past a 16-byte boundary."""
    npd = NP[dt]
    m, n, lda = 301, 517, 531
    A, x, c0 = workloads.gemv_inputs(m, n, seed=8, dist="normal", op_t=bool(op), dtype=npd, lda=lda)
    ref = oracle.gemv(A[:, :n], x, c0, op=op)
    K = n if op == 0 else m
    bnd = gemv_bound(A[:, :n], x, c0, op, K, U64 if dt == 0 else U32)
    big = dev(np.concatenate([np.full(1, np.nan, npd), A.reshape(-1)]))
    for off in (0, 1):
        view = big[off:off + m * lda].reshape(m, lda)[:, :n] if off else dev(A)[:, :n]
        cd = dev(c0)
        sb.sb_gemv(view, dev(x), cd, op=op)
        assert_within(host(cd), ref, bnd, f"offset {off}")


def test_gemv_special_values(sb):
    m, n = 64, 300
    A, x, c0 = workloads.gemv_inputs(m, n, seed=9, dist="normal")
    A[3, 7] = np.inf
    x[7] = 0.0                      # inf * 0 = NaN in row 3
    A[5, 11] = np.nan               # NaN in row 5
    A[9, :] = 1e-310                # subnormal products survive
    x2 = x.copy()
    got = run_gemv(sb, A, x2, c0, 0, 0)
    ref = oracle.gemv(A, x2, c0)
    assert np.isnan(got[3]) and np.isnan(got[5])
    keep = [i for i in range(m) if i not in (3, 5)]
    assert_within(got[keep], ref[keep], gemv_bound(A[keep], x2, c0[keep], 0, n, U64), "specials")
    t = np.zeros((1, 2))
    t[0] = [2.0 ** -1073, 2.0 ** -1073]
    got = run_gemv(sb, t, np.array([0.5, 0.5]), np.zeros(1), 0, 0)
    assert got[0] == 2.0 ** -1074 * 2


def test_gemv_zero_sizes(sb):
    c = dev(np.array([1.5, -2.0]))
    sb.sb_gemv(dev(np.zeros((2, 0))), dev(np.zeros(0)), c)          # n = 0: unchanged
    assert host(c).tolist() == [1.5, -2.0]
    sb.sb_gemv(dev(np.zeros((0, 3))), dev(np.ones(3)), dev(np.zeros(0)))  # m = 0: nothing


@pytest.mark.parametrize("op", [0, 1])
def test_gemv_deterministic(sb, op):
    A, x, c0 = workloads.gemv_inputs(2048, 3000, seed=11, dist="normal", op_t=bool(op))
    Ad, xd = dev(A), dev(x)
    outs = []
    for _ in range(10):
        cd = dev(c0)
        sb.sb_gemv(Ad, xd, cd, op=op)
        outs.append(host(cd))
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


# ------------------------------------------------------------------- DOT ----

@pytest.mark.parametrize("dt", [0, 1])
@pytest.mark.parametrize("n", [1, 2, 3, 255, 256, 257, 4096, 65537, 1000003])
def test_dot_bound(sb, dt, n):
    npd = NP[dt]
    x, y, a0 = workloads.dot_inputs(n, seed=n, dtype=npd)
    ref = oracle.dot(x, y, a0[0])
    ad = dev(a0)
    sb.sb_dot(dev(x), dev(y), ad)
    got = host(ad)[0]
    u = U64 if dt == 0 else U32
    bound = 2 * (n + 1) * u / (1 - (n + 1) * u) * (abs(a0[0]) + float(np.sum(np.abs(x.astype(float) * y))))
    assert abs(got - ref) <= bound


@pytest.mark.parametrize("n", [7, 4096, 1 << 20, (1 << 20) + 5])
def test_dot_integer_exact_and_closed_form(sb, n):
    x, y, a0 = workloads.dot_inputs(n, seed=202, dist="int8")
    ad = dev(a0)
    sb.sb_dot(dev(x), dev(y), ad)
    assert host(ad)[0] == oracle.dot(x, y, a0[0])
    v = np.arange(1, min(n, 1 << 16) + 1, dtype=np.float64)
    ad = dev(np.zeros(1))
    sb.sb_dot(dev(v), dev(v), ad)
    k = v.shape[0]
    assert host(ad)[0] == k * (k + 1) * (2 * k + 1) // 6


def test_dot_misaligned_zero_and_deterministic(sb):
    n = 100003
    x, y, a0 = workloads.dot_inputs(n + 1, seed=4)
    xd, yd = dev(x), dev(y)
    ref = oracle.dot(x[1:], y[:-1], 0.5)
    ad = dev(np.array([0.5]))
    sb.sb_dot(xd[1:], yd[:-1], ad)
    got = host(ad)[0]
    assert abs(got - ref) <= 2 * n * U64 * (0.5 + np.sum(np.abs(x[1:] * y[:-1])))
    z = dev(np.array([3.25]))
    sb.sb_dot(xd[:0], yd[:0], z)
    assert host(z)[0] == 3.25
    vals = set()
    for _ in range(10):
        ad = dev(np.array([0.5]))
        sb.sb_dot(xd[1:], yd[:-1], ad)
        vals.add(host(ad)[0])
    assert len(vals) == 1


# ------------------------------------------------------------------- GER ----

@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("m,n", [(1, 1), (3, 5), (64, 64), (65, 127), (1000, 1531), (4093, 17)])
def test_ger_f64_bitwise(sb, layout, m, n):
    """GER rounds the product and then the sum, as the definition does, so
    the binary64 result equals the oracle bit for bit."""
    x, y, C0 = workloads.ger_inputs(m, n, seed=m + n)
    ref = oracle.ger(x, y, C0)
    Cd = as_layout(C0, layout)
    sb.sb_ger(dev(x), dev(y), Cd)
    assert np.array_equal(host(Cd), ref)


def test_ger_f32_and_misaligned(sb):
    m, n = 513, 1027
    x, y, C0 = workloads.ger_inputs(m, n, seed=3, dtype=np.float32)
    ref = oracle.ger(x, y, C0)
    Cd = dev(C0)
    sb.sb_ger(dev(x), dev(y), Cd)
    got = host(Cd).astype(np.float64)
    bound = 2 * 2 * U32 / (1 - 2 * U32) * (np.abs(C0) + np.abs(np.outer(x, y)))
    assert_within(got, ref, bound, "ger f32")
    # misaligned C (one element past a 16-byte boundary) with padded ldc
    ld = n + 3
    big = np.full(1 + m * ld, np.nan, np.float64)
    Cp = big[1:].reshape(m, ld)
    x, y, C0 = workloads.ger_inputs(m, n, seed=4)
    Cp[:, :n] = C0
    bd = dev(big)
    view = bd[1:].reshape(m, ld)[:, :n]
    sb.sb_ger(dev(x), dev(y), view)
    out = host(bd)[1:].reshape(m, ld)
    assert np.array_equal(out[:, :n], oracle.ger(x, y, C0))
    assert np.isnan(out[:, n:]).all() and np.isnan(host(bd)[0])  # padding untouched


@pytest.mark.parametrize("m,n", [(16384, 1024), (100, 1003), (37, 4096)])
def test_stream_update_probe_leaves_matrix_unchanged(sb, m, n):
    """The GER-pattern probe reads and rewrites C in place: every bit stays."""
    rng = np.random.default_rng(m + n)
    C = rng.standard_normal((m, n))
    Cd = dev(C)
    sb.sb_stream_update(Cd)
    assert np.array_equal(host(Cd).view(np.uint64), C.view(np.uint64))
