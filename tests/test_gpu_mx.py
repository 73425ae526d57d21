"""Microscaled A (OCP MX: E8M0 scale per 32-element block, E4M3 or E2M1
elements) on the GPU against the oracle: the quantiser bit for bit (codes
and scales, including zero, NaN, infinite and subnormal blocks and ragged
widths), the GEMV within the binary32 accumulation bound of the decoded
matrix and exactly where every sum is exact, NaN scales, padded strides,
split rows and the full 16384 x 16384 size with its error against the
binary64 GEMV of the unquantised matrix."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import U32, assert_within, dev, gemv_bound, host, normwise

pytestmark = pytest.mark.gpu

QS = [4, 5]   # MXFP8 (E4M3), MXFP4 (E2M1)


def decode_tables():
    e4 = np.array([oracle.e4m3_to_f32(c) for c in range(256)], dtype=np.float64)
    e2 = np.array([oracle.e2m1_to_f64(c) for c in range(16)], dtype=np.float64)
    x8 = np.array([oracle.e8m0_to_f64(c) for c in range(256)], dtype=np.float64)
    return e4, e2, x8


E4, E2, X8 = decode_tables()


def decode(codes, scales, q, n):
    """The decoded m x n matrix X * P in binary64 (exact)."""
    codes = np.asarray(codes)
    if q == 4:
        P = E4[codes[:, :n]]
    else:
        lo, hi = E2[codes & 15], E2[codes >> 4]
        P = np.empty((codes.shape[0], 2 * codes.shape[1]))
        P[:, 0::2], P[:, 1::2] = lo, hi
        P = P[:, :n]
    X = np.repeat(X8[np.asarray(scales)], 32, axis=1)[:, :n]
    return X * P


def to_device_mx(sb, codes, scales, q, n, pad_q=0, pad_s=0, fill=0):
    m = codes.shape[0]
    Q, S = sb.mx_buffers(q, m, n)
    if pad_q or pad_s or fill:
        Q = torch.full((m, Q.shape[1] + pad_q), fill, dtype=torch.uint8, device="cuda")
        S = torch.full((m, S.shape[1] + pad_s), fill, dtype=torch.uint8, device="cuda")
    Q[:, :codes.shape[1]] = dev(codes)
    S[:, :scales.shape[1]] = dev(scales)
    return Q, S


def gpu_quantize(sb, A, q):
    m, n = A.shape
    Q, S = sb.mx_buffers(q, m, n)
    sb.sb_quantize_mx(dev(A), Q, S, q)
    rb = oracle.mx_row_bytes(q, n)
    return host(Q)[:, :rb], host(S)[:, :(n + 31) // 32]


SHAPES = [(1, 1), (3, 31), (5, 33), (2, 64), (17, 1000), (64, 4097), (9, 40001)]


@pytest.mark.parametrize("q", QS)
@pytest.mark.parametrize("m,n", SHAPES)
def test_quantize_mx_bitwise(sb, q, m, n):
    rng = np.random.default_rng(m * 7 + n)
    A = (rng.standard_normal((m, n)) * 2.0 ** rng.integers(-40, 40, (m, 1))).astype(np.float32)
    if n >= 64 and m >= 2:
        A[0, 32:64] = 0.0
        A[1, :32] = np.float32(1.5e-42)        # a subnormal block
    if n >= 200 and m >= 5:
        A[2, 70] = np.nan
        A[3, 130] = -np.inf
        A[4, 140:160] = -0.0
    codes, scales = oracle.quantize_mx(A, q)
    gq, gs = gpu_quantize(sb, A, q)
    assert np.array_equal(gs, scales)
    assert np.array_equal(gq, codes)


@pytest.mark.parametrize("q", QS)
def test_quantize_mx_ties_and_saturation(sb, q):
    """Values placed on every rounding boundary of the element format, and
    beyond its largest value, in a block whose scale is 1 (amax in the
    format's top binade)."""
    top = 448.0 if q == 4 else 6.0
    if q == 4:
        vals = np.array([oracle.e4m3_to_f32(c) for c in range(0, 127)], dtype=np.float64)
    else:
        vals = E2[:8]
    mids = (vals[1:] + vals[:-1]) / 2
    cand = np.concatenate([mids, -mids, [top, top * 1.05, -top * 1.1, 0.0, -0.0]])
    n = 32 * ((len(cand) + 30) // 31)
    A = np.zeros((1, n), dtype=np.float32)
    for b in range(n // 32):
        chunk = cand[31 * b:31 * b + 31]
        A[0, 32 * b] = top                     # sets the block's scale to 2^0
        A[0, 32 * b + 1:32 * b + 1 + len(chunk)] = chunk
    codes, scales = oracle.quantize_mx(A, q)
    assert (scales == 127).all()
    gq, gs = gpu_quantize(sb, A, q)
    assert np.array_equal(gq, codes) and np.array_equal(gs, scales)


def run_gemv_mx(sb, codes, scales, q, x, c0, **pad):
    n = x.shape[0]
    Q, S = to_device_mx(sb, codes, scales, q, n, **pad)
    cd = dev(c0.astype(np.float32))
    sb.sb_gemv_mx(Q, S, dev(x), cd, q)
    return host(cd).astype(np.float64)


@pytest.mark.parametrize("q", QS)
@pytest.mark.parametrize("m,n", [(1, 7), (3, 32), (40, 1000), (257, 4096), (70, 33000), (1000, 777),
                                 (37, 10241), (9, 20483)])   # x just above 40 KiB and 80 KiB
def test_gemv_mx_bound(sb, q, m, n):
    A, x, c0 = workloads.gemv_inputs(m, n, seed=m + 3 * n, dist="normal", dtype=np.float32)
    codes, scales = oracle.quantize_mx(A, q)
    ref = oracle.gemv_mx(codes, scales, x, c0, q, n)
    got = run_gemv_mx(sb, codes, scales, q, x, c0)
    D = decode(codes, scales, q, n)
    assert_within(got, ref, gemv_bound(D, x, c0, 0, n, U32), f"gemv_mx q={q} {m}x{n}")
    got2 = run_gemv_mx(sb, codes, scales, q, x, c0, pad_q=48, pad_s=5)   # padded strides
    assert np.array_equal(got, got2)


@pytest.mark.parametrize("q", QS)
@pytest.mark.parametrize("m,n", [(5, 4097), (17, 8191), (3, 16385), (9, 16415), (130, 70001)])
def test_gemv_mx_row_edges_ignore_padding(sb, q, m, n):
    """Rows that end inside a 16-byte code vector, with every padding byte of
    Q and S set to 0xFF (a NaN E4M3 code, a NaN E8M0 scale): the padding
    never reaches the result, which equals the zero-padded run bit for bit
    and lies within the bound of the oracle."""
    A, x, c0 = workloads.gemv_inputs(m, n, seed=n, dist="normal", dtype=np.float32)
    codes, scales = oracle.quantize_mx(A, q)
    ref = oracle.gemv_mx(codes, scales, x, c0, q, n)
    got = run_gemv_mx(sb, codes, scales, q, x, c0, pad_q=32, pad_s=3)
    poisoned = run_gemv_mx(sb, codes, scales, q, x, c0, pad_q=32, pad_s=3, fill=0xFF)
    assert np.array_equal(got, poisoned)
    D = decode(codes, scales, q, n)
    assert_within(got, ref, gemv_bound(D, x, c0, 0, n, U32), f"gemv_mx q={q} {m}x{n}")


@pytest.mark.parametrize("q", QS)
def test_gemv_mx_exact_integers(sb, q):
    """Codes of small integers and halves, scales 2^-2 .. 2^1, integer x:
    every product and partial sum is exact in binary32, so any order gives
    the oracle's bits."""
    rng = np.random.default_rng(q)
    m, n = 300, 5000
    if q == 4:
        pool = [c for c in range(256) if np.isfinite(E4[c]) and abs(E4[c]) <= 8 and (2 * E4[c]) % 1 == 0]
        codes = rng.choice(pool, (m, n)).astype(np.uint8)
    else:
        codes = rng.integers(0, 256, (m, (n + 1) // 2)).astype(np.uint8)
        codes[:, -1] &= 0x0F if n % 2 else 0xFF
    scales = rng.integers(125, 129, (m, (n + 31) // 32)).astype(np.uint8)
    x = rng.integers(-8, 9, n).astype(np.float32)
    c0 = rng.integers(-100, 100, m).astype(np.float64)
    ref = oracle.gemv_mx(codes, scales, x, c0, q, n)
    got = run_gemv_mx(sb, codes, scales, q, x, c0)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("q", QS)
def test_gemv_mx_nan_scale(sb, q):
    m, n = 4, 100
    A, x, c0 = workloads.gemv_inputs(m, n, seed=5, dist="normal", dtype=np.float32)
    A[2, 40] = np.nan
    codes, scales = oracle.quantize_mx(A, q)
    assert scales[2, 1] == 255
    got = run_gemv_mx(sb, codes, scales, q, x, c0)
    assert np.isnan(got[2]) and np.isfinite(got[[0, 1, 3]]).all()


@pytest.mark.parametrize("q", QS)
def test_mx_full_size(sb, q):
    """16384 x 16384: GPU quantiser against the oracle on every code and
    scale, GEMV against the oracle within the bound, and the error of the
    whole precision form against the binary64 GEMV of the unquantised A."""
    m = n = 16384
    g = torch.Generator(device="cuda")
    g.manual_seed(601)
    Ad = torch.randn((m, n), generator=g, device="cuda", dtype=torch.float32)
    A = host(Ad)
    Q, S = sb.mx_buffers(q, m, n)
    sb.sb_quantize_mx(Ad, Q, S, q)
    codes, scales = oracle.quantize_mx(A, q)
    rb = oracle.mx_row_bytes(q, n)
    assert np.array_equal(host(S), scales) and np.array_equal(host(Q)[:, :rb], codes)
    del Ad
    rng = np.random.default_rng(602)
    x = rng.standard_normal(n).astype(np.float32)
    c0 = np.zeros(m)
    cd = torch.zeros(m, dtype=torch.float32, device="cuda")
    sb.sb_gemv_mx(Q, S, dev(x), cd, q)
    got = host(cd).astype(np.float64)
    ref = oracle.gemv_mx(codes, scales, x, c0, q, n)
    D = decode(codes, scales, q, n)
    assert_within(got, ref, gemv_bound(D, x, c0, 0, n, U32), "full")
    exact = oracle.gemv(A.astype(np.float64), x.astype(np.float64), c0)
    err = normwise(got, exact)
    print(f"q={q}: normwise error against the binary64 GEMV of A: {err:.3e}")
    assert err < (0.04 if q == 4 else 0.15)


@pytest.mark.parametrize("q", QS)
def test_mx_padded_strides_and_specials(sb, q):
    """A read through a padded leading dimension into padded Q and S rows;
    an infinite x entry and a NaN in A propagate as in the oracle."""
    m, n, lda = 37, 1001, 1040
    rng = np.random.default_rng(70 + q)
    store = np.full((m, lda), np.nan, dtype=np.float32)
    store[:, :n] = rng.standard_normal((m, n)).astype(np.float32)
    A = np.ascontiguousarray(store[:, :n])
    codes, scales = oracle.quantize_mx(A, q)
    Q = torch.zeros((m, 16 * ((oracle.mx_row_bytes(q, n) + 15) // 16) + 64), dtype=torch.uint8, device="cuda")
    S = torch.zeros((m, (n + 31) // 32 + 7), dtype=torch.uint8, device="cuda")
    sb.sb_quantize_mx(dev(store)[:, :n], Q, S, q)
    rb, nb = oracle.mx_row_bytes(q, n), (n + 31) // 32
    assert np.array_equal(host(Q)[:, :rb], codes) and np.array_equal(host(S)[:, :nb], scales)
    x = rng.standard_normal(n).astype(np.float32)
    x[500] = np.inf
    c0 = np.zeros(m)
    cd = torch.zeros(m, dtype=torch.float32, device="cuda")
    sb.sb_gemv_mx(Q, S, dev(x), cd, q)
    got = host(cd).astype(np.float64)
    ref = oracle.gemv_mx(codes, scales, x, c0, q, n)
    assert np.array_equal(np.isnan(got), np.isnan(ref)) and np.array_equal(np.isinf(got), np.isinf(ref))
    fin = np.isfinite(ref)
    assert fin.sum() < m and (~fin).sum() > 0
