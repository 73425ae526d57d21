"""Two-sided GEMV (c += A x and d += A^T y in one pass over A) against the
oracle: integer data bit for bit, random data within the GEMV bound for
each output, every band configuration of the kernel (direct update, row
bands only, column bands only, both), both layouts, padded and misaligned
storage, aliased inputs, empty shapes and the full 16384 x 16384 size."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import U32, U64, assert_within, dev, gemv_bound, host

pytestmark = pytest.mark.gpu

NP = {0: np.float64, 1: np.float32}


def inputs(m, n, seed, dist, npd):
    A, x, c0 = workloads.gemv_inputs(m, n, seed=seed, dist=dist, dtype=npd)
    rng = np.random.default_rng(seed + 1)
    if dist in ("int8", "int7"):
        k = 8 if dist == "int8" else 7
        y = rng.integers(-k, k + 1, m).astype(npd)
        d0 = rng.integers(-k, k + 1, n).astype(npd)
    else:
        y = rng.standard_normal(m).astype(npd)
        d0 = rng.standard_normal(n).astype(npd)
    return A, x, y, c0, d0


def as_layout(A, layout):
    return dev(A) if layout == 0 else dev(np.ascontiguousarray(A.T)).t()


def run(sb, A, x, y, c0, d0, layout):
    cd, dd = dev(c0), dev(d0)
    sb.sb_gemv2(as_layout(A, layout), dev(x), dev(y), cd, dd)
    return host(cd), host(dd)


SHAPES = [(1, 1), (1, 7), (7, 1), (8, 8), (9, 130), (64, 64), (130, 9), (1000, 1531), (4093, 129),
          (129, 4093), (300, 40000), (20000, 300), (2049, 2047)]


@pytest.mark.parametrize("dt", [0, 1])
@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("m,n", SHAPES)
def test_gemv2_bound_and_integer(sb, dt, layout, m, n):
    npd = NP[dt]
    u = U64 if dt == 0 else U32
    A, x, y, c0, d0 = inputs(m, n, m * 31 + n, "normal", npd)
    cref, dref = oracle.gemv2(A, x, y, c0, d0)
    c, d = run(sb, A, x, y, c0, d0, layout)
    assert_within(c, cref, gemv_bound(A, x, c0, 0, n, u), f"c {m}x{n}")
    assert_within(d, dref, gemv_bound(A, y, d0, 1, m, u), f"d {m}x{n}")
    Ai, xi, yi, ci, di = inputs(m, n, 3, "int7" if dt else "int8", npd)
    if dt == 0 or max(m, n) * 49 < 1 << 24:
        c, d = run(sb, Ai, xi, yi, ci, di, layout)
        cref, dref = oracle.gemv2(Ai, xi, yi, ci, di)
        assert np.array_equal(c, cref) and np.array_equal(d, dref)


def test_gemv2_deterministic_and_layout_symmetry(sb):
    """Runs repeat bit for bit; (row-major, A) and (column-major, A^T) on the
    same buffer compute the same sums with the roles of the outputs swapped."""
    m, n = 3001, 2500
    A, x, y, c0, d0 = inputs(m, n, 17, "uniform", np.float64)
    Ad = dev(A)
    outs = []
    for _ in range(3):
        cd, dd = dev(c0), dev(d0)
        sb.sb_gemv2(Ad, dev(x), dev(y), cd, dd)
        outs.append((host(cd), host(dd)))
    assert all(np.array_equal(outs[0][0], o[0]) and np.array_equal(outs[0][1], o[1]) for o in outs)
    # A^T as a column-major n x m view of the same storage: c' += A^T y, d' += A x
    cd, dd = dev(d0), dev(c0)
    sb.sb_gemv2(Ad.t(), dev(y), dev(x), cd, dd)
    assert np.array_equal(host(cd), outs[0][1]) and np.array_equal(host(dd), outs[0][0])


def test_gemv2_padded_misaligned_aliased(sb):
    m, n, lda = 777, 1001, 1003
    A, x, _ = workloads.gemv_inputs(m, n, seed=9, dist="normal", lda=lda)
    Av = np.ascontiguousarray(A[:, :n])
    rng = np.random.default_rng(9)
    y, c0, d0 = rng.standard_normal(m), rng.standard_normal(m), rng.standard_normal(n)
    cref, dref = oracle.gemv2(Av, x, y, c0, d0)
    store = dev(A)                                     # NaN padding beyond column n
    cd, dd = dev(c0), dev(d0)
    sb.sb_gemv2(store[:, :n], dev(x), dev(y), cd, dd)
    assert_within(host(cd), cref, gemv_bound(Av, x, c0, 0, n, U64), "padded c")
    assert_within(host(dd), dref, gemv_bound(Av, y, d0, 1, m, U64), "padded d")
    flat = dev(np.concatenate([[0.0], Av.ravel()]))
    cd, dd = dev(c0), dev(d0)
    sb.sb_gemv2(flat[1:].view(m, n), dev(x), dev(y), cd, dd)   # base off 16-byte alignment
    assert_within(host(cd), cref, gemv_bound(Av, x, c0, 0, n, U64), "misaligned c")
    assert_within(host(dd), dref, gemv_bound(Av, y, d0, 1, m, U64), "misaligned d")
    # square matrix, x and y the same tensor
    S, v, c0s = workloads.gemv_inputs(900, 900, seed=10)
    d0s = np.zeros(900)
    vd = dev(v)
    cd, dd = dev(c0s), dev(d0s)
    sb.sb_gemv2(dev(S), vd, vd, cd, dd)
    cref, dref = oracle.gemv2(S, v, v, c0s, d0s)
    assert_within(host(cd), cref, gemv_bound(S, v, c0s, 0, 900, U64), "aliased c")
    assert_within(host(dd), dref, gemv_bound(S, v, d0s, 1, 900, U64), "aliased d")


def test_gemv2_empty(sb):
    c = dev(np.array([1.5, 2.5]))
    d = dev(np.zeros(0))
    sb.sb_gemv2(torch.zeros((2, 0), dtype=torch.float64, device="cuda"), dev(np.zeros(0)),
                dev(np.ones(2)), c, d)
    assert np.array_equal(host(c), [1.5, 2.5])
    d = dev(np.array([4.0, 5.0, 6.0]))
    sb.sb_gemv2(torch.zeros((0, 3), dtype=torch.float64, device="cuda"), dev(np.ones(3)),
                dev(np.zeros(0)), dev(np.zeros(0)), d)
    assert np.array_equal(host(d), [4.0, 5.0, 6.0])


@pytest.mark.parametrize("m,n", [(16384, 16384), (262144, 256), (256, 262144)])
def test_gemv2_full_sizes(sb, m, n):
    """The sizes of the measured workload, every entry against the oracle."""
    A, x, c0 = workloads.gemv_inputs(m, n, seed=201)
    rng = np.random.default_rng(202)
    y, d0 = rng.uniform(-1, 1, m), rng.uniform(-1, 1, n)
    cref, dref = oracle.gemv2(A, x, y, c0, d0)
    c, d = run(sb, A, x, y, c0, d0, 0)
    assert_within(c, cref, gemv_bound(A, x, c0, 0, n, U64), "full c")
    assert_within(d, dref, gemv_bound(A, y, d0, 1, m, U64), "full d")


def test_gemv2_specials_propagate(sb):
    """NaN and infinity reach exactly the outputs whose sums contain them,
    as in the oracle: entries of A poison one row sum and one column sum;
    an infinite x entry every row sum, a NaN y entry every column sum."""
    m, n = 300, 500
    A, x, y, c0, d0 = inputs(m, n, 77, "normal", np.float64)
    A[10, 20] = np.nan
    A[30, 40] = np.inf

    def same_specials(got, ref):
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        assert np.array_equal(np.isposinf(got), np.isposinf(ref))
        assert np.array_equal(np.isneginf(got), np.isneginf(ref))

    cref, dref = oracle.gemv2(A, x, y, c0, d0)
    for layout in (0, 1):
        c, d = run(sb, A, x, y, c0, d0, layout)
        same_specials(c, cref)
        same_specials(d, dref)
        assert np.isfinite(cref).sum() == m - 2 and np.isfinite(dref).sum() == n - 2
    x2, y2 = x.copy(), y.copy()
    x2[100], y2[200] = -np.inf, np.nan
    cref, dref = oracle.gemv2(A, x2, y2, c0, d0)
    c, d = run(sb, A, x2, y2, c0, d0, 0)
    same_specials(c, cref)
    same_specials(d, dref)
