"""Host-side parts of the serving loop: the trace generator and the
first-fit HBM pool (no GPU needed)."""
import math

import numpy as np

from paper_2108_02025_amd.serve import Pool, device_bytes, make_trace


def test_trace_statistics():
    tr = make_trace(4096, rate=1e5, seed=501)
    arr = np.array([r.arrival for r in tr])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    gaps = np.diff(arr)
    assert abs(gaps.mean() * 1e5 - 1) < 0.05              # mean inter-arrival 1/rate
    m = np.array([r.m for r in tr])
    n = np.array([r.n for r in tr])
    assert m.min() >= 64 and m.max() <= 8192 and n.min() >= 64 and n.max() <= 8192
    lm = np.log(m)
    assert abs(lm.mean() - (math.log(64) + math.log(8192)) / 2) < 0.1  # log-uniform
    frac = np.mean([r.kind == "bf16" for r in tr])
    assert 0.45 < frac < 0.55
    assert len({r.seed for r in tr}) == len(tr)
    assert make_trace(8, seed=1)[3].m == make_trace(8, seed=1)[3].m


def test_pool_first_fit_and_merge():
    p = Pool(1 << 20)
    a = p.alloc(1000)
    b = p.alloc(5000)
    c = p.alloc(300)
    assert (a, b) == (0, 1024) and c == 1024 + 5120
    assert p.alloc(1 << 20) is None                          # too big while others live
    p.free(b, 5000)
    assert p.alloc(4000) == 1024                             # first fit reuses the hole
    p.free(a, 1000)
    p.free(1024, 4000)
    p.free(c, 300)
    assert p.free_list == [(0, 1 << 20)] and p.used == 0     # everything merged back
    assert p.alloc(1 << 20) == 0


def test_request_bytes():
    assert device_bytes("f32", 64, 64) == 64 * 64 * 4 + 256 + 256
    assert device_bytes("bf16", 100, 100) == 20224 + 512 + 512 + 512


def test_trace_dot_requests():
    from paper_2108_02025_amd.serve import make_trace
    base = make_trace(300, seed=3)
    mixed = make_trace(300, seed=3, dot_fraction=0.3, dot_hi=1 << 16)
    dots = [r for r in mixed if r.op == "dot"]
    assert 50 < len(dots) < 130
    assert all(r.m == 1 and r.kind == "f32" and 64 <= r.n <= 1 << 16 for r in dots)
    for a, b in zip(base, mixed):   # the GEMV fields are drawn first and do not change
        assert a.arrival == b.arrival
        if b.op == "gemv":
            assert (a.kind, a.m, a.n, a.seed) == (b.kind, b.m, b.n, b.seed)
    assert all(r.op == "gemv" for r in base)
