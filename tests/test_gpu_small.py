"""Small-problem paths (the single-launch forms of section 4.3's
Algorithm 3 and of a GEMV-T whose row split would be at most four ways):
parity with the oracle on both sides of each cutoff, integer exactness,
misaligned bases and repeat-run determinism.  The cutoffs are read from
the library's workspace sizes (a path that needs no workspace is the
single-launch one), so the tests follow the library's plan."""
import numpy as np
import pytest
import torch

import oracle
import dot2_tree
import workloads
from gpu_util import U32, U64, assert_within, dev, gamma, gemv_bound, host

pytestmark = pytest.mark.gpu

NP = {0: np.float64, 1: np.float32}


def dot_cutoff(sb, kind, dt):
    """Largest n whose DOT needs no workspace (the single-workgroup path)."""
    lo, hi = 1, 1 << 24
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if sb.sb_workspace_bytes(kind, dt, 0, 0, 1, mid) == 0:
            lo = mid
        else:
            hi = mid - 1
    return lo


def dot_check(sb, x, y, a0, dt):
    ad = dev(np.array([a0], NP[dt]))
    sb.sb_dot(dev(x), dev(y), ad)
    got = float(host(ad)[0])
    ref = oracle.dot(x, y, a0)
    n = x.shape[0]
    u = U64 if dt == 0 else U32
    bound = 2 * gamma(n + 1, u) * (abs(a0) + float(np.sum(np.abs(x.astype(float) * y))))
    assert abs(got - ref) <= bound, (n, got, ref, bound)
    return got


@pytest.mark.parametrize("dt", [0, 1])
def test_dot_across_cutoff(sb, dt):
    kind = sb.SB_KIND_DOT
    cut = dot_cutoff(sb, kind, dt)
    assert cut * 2 * (8 if dt == 0 else 4) >= 64 * 1024   # the cutoff is not degenerate
    for n in (cut - 1, cut, cut + 1, cut + 17):
        x, y, a0 = workloads.dot_inputs(n, seed=n, dtype=NP[dt])
        dot_check(sb, x, y, float(a0[0]), dt)
        xi, yi, ai = workloads.dot_inputs(n, seed=7, dist="int7" if dt else "int8", dtype=NP[dt])
        if dt == 0 or n * 49 < 1 << 24:
            ad = dev(ai)
            sb.sb_dot(dev(xi), dev(yi), ad)
            assert host(ad)[0] == oracle.dot(xi, yi, ai[0])


@pytest.mark.parametrize("dt", [0, 1])
def test_dot_small_misaligned_and_deterministic(sb, dt):
    n = 5001
    x, y, a0 = workloads.dot_inputs(n + 1, seed=31, dtype=NP[dt])
    xd, yd = dev(x), dev(y)
    vals = set()
    for _ in range(5):
        ad = dev(np.array([0.25], NP[dt]))
        sb.sb_dot(xd[1:], yd[:-1], ad)
        vals.add(float(host(ad)[0]))
    assert len(vals) == 1
    ref = oracle.dot(x[1:], y[:-1], 0.25)
    u = U64 if dt == 0 else U32
    assert abs(vals.pop() - ref) <= 2 * gamma(n + 1, u) * (0.25 + float(np.sum(np.abs(x[1:].astype(float) * y[:-1]))))


def test_dot2_across_cutoff(sb):
    cut = dot_cutoff(sb, sb.SB_KIND_DOT2, 1)
    for n in (cut, cut + 1):
        x, y, _, _ = workloads.illcond_dot_inputs(n, seed=n)
        ad = dev(np.array([0.75], np.float32))
        sb.sb_dot2_f32(dev(x), dev(y), ad)
        got = float(host(ad)[0])
        ex = oracle.dot_exact_f32(x, y, 0.75)
        ab = oracle.dot_exact_f32(x, y, 0.75, absval=True)
        g = gamma(dot2_tree.path_length(n), U32)
        # Dot2's bound (Ogita, Rump and Oishi): u|s| + gamma_L^2 sum|x y| with
        # L the launch's longest addition path, plus the final rounding to binary32
        assert abs(got - ex) <= 2 * U32 * abs(ex) + g * g * ab, (n, got, ex)


# GEMV-T (row-major c += A^T x, column-major c += A x) whose row split
# would be two ways (128..191 rows) runs unsplit; the others keep their plan.
T_SHAPES = [(128, 16384), (191, 16383), (150, 3001), (130, 257), (160, 1), (64, 16384), (63, 5000),
            (100, 1), (192, 4096), (1024, 1024)]


@pytest.mark.parametrize("dt", [0, 1])
@pytest.mark.parametrize("rows,cols", T_SHAPES)
def test_gemv_t_small_path(sb, dt, rows, cols):
    npd = NP[dt]
    u = U64 if dt == 0 else U32
    A, x, c0 = workloads.gemv_inputs(rows, cols, seed=rows + cols, dist="normal", op_t=True, dtype=npd)
    ref = oracle.gemv(A, x, c0, op=1)
    Ad, xd = dev(A), dev(x)
    outs = []
    for _ in range(2):
        cd = dev(c0)
        sb.sb_gemv(Ad, xd, cd, op=1)
        outs.append(host(cd))
    assert np.array_equal(outs[0], outs[1])
    assert_within(outs[0], ref, gemv_bound(A, x, c0, 1, rows, u), f"T {rows}x{cols}")
    # column-major c += A x on the same buffer is the same kernel: same bits
    # (a single column has unit strides both ways and is read as row-major)
    cd = dev(c0)
    sb.sb_gemv(Ad.t(), xd, cd, op=0)
    if cols > 1:
        assert np.array_equal(host(cd), outs[0])
    else:
        assert_within(host(cd), ref, gemv_bound(A, x, c0, 1, rows, u), "one column")
    Ai, xi, ci = workloads.gemv_inputs(rows, cols, seed=5, dist="int7" if dt else "int8", op_t=True, dtype=npd)
    cd = dev(ci)
    sb.sb_gemv(dev(Ai), dev(xi), cd, op=1)
    assert np.array_equal(host(cd), oracle.gemv(Ai, xi, ci, op=1))


@pytest.mark.parametrize("dt", [0, 1])
def test_cutoff_override_changes_path_not_result(sb, dt):
    """Forcing each path through the handle's cutoffs gives results within
    the same bound; the default handle is restored afterwards."""
    h = sb.handle_for(torch.empty(1, device="cuda"))
    npd = NP[dt]
    u = U64 if dt == 0 else U32
    x, y, a0 = workloads.dot_inputs(50000, seed=3, dtype=npd)
    A, xt, c0 = workloads.gemv_inputs(600, 2000, seed=4, dist="normal", op_t=True, dtype=npd)
    dref, tref = oracle.dot(x, y, a0[0]), oracle.gemv(A, xt, c0, op=1)
    keep = [sb.sb_get_cutoff(k, h) for k in (0, 1)]
    try:
        for dot_cut, t_cut in ((0, 0), (1 << 40, 64)):
            sb.sb_set_cutoff(0, dot_cut, h)
            sb.sb_set_cutoff(1, t_cut, h)
            ad = dev(a0)
            sb.sb_dot(dev(x), dev(y), ad)
            bound = 2 * gamma(50001, u) * (abs(a0[0]) + float(np.sum(np.abs(x.astype(float) * y))))
            assert abs(float(host(ad)[0]) - dref) <= bound
            cd = dev(c0)
            sb.sb_gemv(dev(A), dev(xt), cd, op=1)
            assert_within(host(cd), tref, gemv_bound(A, xt, c0, 1, 600, u), f"cutoffs {dot_cut} {t_cut}")
    finally:
        sb.sb_set_cutoff(0, keep[0], h)
        sb.sb_set_cutoff(1, keep[1], h)


def test_gemv_t_small_padded_and_misaligned(sb):
    rows, cols, lda = 150, 1001, 1003
    A, x, c0 = workloads.gemv_inputs(rows, cols, seed=9, dist="normal", op_t=True, lda=lda)
    store = dev(A)                                   # rows x lda, NaN padding beyond cols
    ref = oracle.gemv(np.ascontiguousarray(A[:, :cols]), x, c0, op=1)
    cd = dev(c0)
    sb.sb_gemv(store[:, :cols], dev(x), cd, op=1)
    assert_within(host(cd), ref, gemv_bound(A[:, :cols], x, c0, 1, rows, U64), "padded")
    flat = dev(np.concatenate([[0.0], A[:, :cols].ravel()]))
    Am = flat[1:].view(rows, cols)                   # base 8 bytes off 16-byte alignment
    cd = dev(c0)
    sb.sb_gemv(Am, dev(x), cd, op=1)
    assert_within(host(cd), ref, gemv_bound(A[:, :cols], x, c0, 1, rows, U64), "misaligned")
