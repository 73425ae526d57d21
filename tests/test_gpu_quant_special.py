"""The GPU row quantiser on rows holding NaN, infinities, signed zeros and
subnormal magnitudes: scales and codes bit for bit equal to the CPU oracle
and to the values written by hand from the per-row scale rule
(tests/golden/quantize_special_rows.txt), for bfloat16 and E4M3."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host
from goldens import quantize_special_rows

pytestmark = pytest.mark.gpu

FMT = {"bf16": (2, torch.int16, np.uint16, oracle.Q_BF16), "e4m3": (3, torch.uint8, np.uint8, oracle.Q_E4M3)}


def gpu_quantize(sb, A, fmt):
    q, tdt, ndt, _ = FMT[fmt]
    m, n = A.shape
    Aq = torch.empty((m, n), dtype=tdt, device="cuda")
    s = torch.empty(m, dtype=torch.float32, device="cuda")
    sb.sb_quantize_rows(dev(A), Aq, s, q)
    return host(Aq).view(ndt), host(s)


@pytest.mark.parametrize("fmt", ["bf16", "e4m3"])
def test_quantiser_special_rows_match_hand_values(sb, fmt):
    rows, exp = quantize_special_rows()
    want_s, want_q = exp[fmt]
    # the five entries spread over the 256 threads of a row's workgroup,
    # inside rows of zeros (which change neither amax nor the other codes)
    n = 1000
    pos = [0, 255, 256, 511, 999]
    A = np.zeros((rows.shape[0], n), np.float32)
    A[:, pos] = rows
    codes, s = gpu_quantize(sb, A, fmt)
    assert np.array_equal(s.view(np.uint32), want_s), (s.view(np.uint32), want_s)
    assert np.array_equal(codes[:, pos], want_q), (codes[:, pos], want_q)
    rest = np.ones(n, bool)
    rest[pos] = False
    assert not codes[:, rest].any()
    codes_o, s_o = oracle.quantize_rows(A, FMT[fmt][3])
    assert np.array_equal(codes, codes_o) and np.array_equal(s.view(np.uint32), s_o.view(np.uint32))


@pytest.mark.parametrize("fmt", ["bf16", "e4m3"])
def test_quantiser_planted_specials_bitwise(sb, fmt):
    """Random normal rows with NaN, +-inf and -0 planted at random places,
    rows scaled into the subnormal range (amax from 2^-149 up to the smallest
    normal) and rows of huge magnitude: codes and scales bit for bit equal to
    the oracle's."""
    rng = np.random.default_rng(2024)
    m, n = 512, 4099
    A = rng.standard_normal((m, n)).astype(np.float32)
    for i in range(0, m, 7):
        k = int(rng.integers(1, 6))
        cols = rng.integers(0, n, k)
        A[i, cols] = rng.choice(np.array([np.nan, np.inf, -np.inf, -0.0], np.float32), k)
    sub = np.arange(3, m, 11)
    A[sub] *= np.exp2(-rng.integers(126, 152, sub.size)).astype(np.float32)[:, None]
    A[5::13] *= np.float32(2.0 ** 100)
    A[9] = np.nan
    A[10] = 0.0
    codes, s = gpu_quantize(sb, A, fmt)
    codes_o, s_o = oracle.quantize_rows(A, FMT[fmt][3])
    assert np.array_equal(s.view(np.uint32), s_o.view(np.uint32))
    bad = np.argwhere(codes != codes_o)
    assert bad.size == 0, f"{len(bad)} codes differ; first at {bad[0].tolist()}"
