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


# ------------------------------------------------------- scheduler policy ----
# The library's Scheduler driven by a simulated clock and a test-only device
# model (tests/serve_sim.py), which also asserts that no batch starts before
# its requests are generated and that live operand blocks never overlap or
# leave the budget.

from serve_sim import run_sim  # noqa: E402


def _trace(n, rate, seed, lo=64, hi=8192):
    tr = make_trace(n, rate=rate, seed=seed, lo=lo, hi=hi)
    return np.array([r.arrival for r in tr]), np.array([r.device_bytes for r in tr], dtype=np.int64)


def test_scheduler_admission_under_budget_and_slot_reuse():
    arr, db = _trace(300, 5e4, 7, hi=2048)
    budget = 24 << 20
    sched, ex = run_sim(arr, db, budget)
    assert (sched.status == 1).all()
    assert sched.pool.used == 0 and sched.pool.free_list == [(0, budget)]
    assert sched.max_queue > 5                        # the small budget made requests queue
    assert sched.batches > 10 and not ex.live
    # memory was reused: the 300 requests need many budgets' worth in total
    assert db.sum() > 10 * budget


def test_scheduler_fifo_no_starvation():
    """A request needing most of the budget, behind small ones and followed
    by a steady stream of small ones, is admitted before every request that
    arrived after it: admission never skips the queue head."""
    arr, db = _trace(400, 1e5, 11, hi=1024)
    budget = 32 << 20
    db[20] = 30 << 20
    sched, ex = run_sim(arr, db, budget)
    assert (sched.status == 1).all()
    order = np.argsort(sched.t_admit, kind="stable")
    assert (np.diff(sched.t_admit) >= 0).all()        # admitted in arrival order
    assert sched.t_admit[20] <= sched.t_admit[21:].min()
    assert sched.t_done[20] < np.inf and order[20] == 20


def test_scheduler_rejects_requests_larger_than_the_budget():
    arr, db = _trace(50, 2e4, 3, hi=1024)
    budget = 8 << 20
    db[[4, 30]] = budget + 256
    sched, ex = run_sim(arr, db, budget)
    assert list(np.flatnonzero(sched.status == 2)) == [4, 30]
    assert np.isinf(sched.t_done[[4, 30]]).all() and np.isnan(ex.gen_end[[4, 30]]).all()
    assert (np.delete(sched.status, [4, 30]) == 1).all()


def test_scheduler_deadlines_and_cancellation():
    """A burst that the budget cannot admit at once: requests whose deadline
    passes while they wait leave unserved, cancelled ones too, and neither
    kind is ever generated; the rest are served."""
    n = 200
    arr = np.zeros(n)
    db = np.full(n, 4 << 20, dtype=np.int64)
    budget = 16 << 20                                  # four requests at a time
    deadlines = np.full(n, np.inf)
    deadlines[100:] = 200e-6                           # the later half must be admitted within 200 us
    sched, ex = run_sim(arr, db, budget, deadlines=deadlines, cancel_at={50e-6: [10, 11, 150]})
    expired = np.flatnonzero(sched.status == 3)
    assert {10, 11}.issubset(expired) and 150 in expired
    assert (sched.status[100:] == 3).sum() > 90        # most of the later half expired
    assert np.isnan(ex.gen_end[expired]).all()         # never generated
    assert (sched.t_admit[sched.status == 1] <= np.where(np.isfinite(deadlines), deadlines, np.inf)[
        sched.status == 1]).all()
    assert ((sched.status == 1) | (sched.status == 3)).all()
    assert sched.pool.used == 0


def test_scheduler_backlog_drains_and_caps_hold():
    """A burst of 800 requests at once, then a steady 1e5/s: the backlog
    drains (the last quarter of the trace is served near the steady-state
    latency), no admission round exceeds max_round_bytes and no batch
    exceeds max_batch_bytes (beyond a single request that is larger)."""
    arr, db = _trace(3000, 1e5, 501)
    arr[:800] = 0.0
    budget = 4 << 30
    caps = dict(max_round_bytes=256 << 20, max_batch_bytes=512 << 20)
    sched, ex = run_sim(arr, db, budget, **caps)
    assert (sched.status == 1).all()
    lat = sched.t_done - arr
    assert np.median(lat[-750:]) < 1e-3 and np.median(lat[:800]) > 2 * np.median(lat[-750:])
    for start, end, ids in ex.batches:
        assert len(ids) == 1 or db[ids].sum() <= caps["max_batch_bytes"]
    rounds = {}
    for i, r in enumerate(sched.round_of):
        rounds.setdefault(int(r), []).append(i)
    assert all(len(v) == 1 or db[v].sum() <= caps["max_round_bytes"] for v in rounds.values())


def test_scheduler_overload_throughput_beats_waiting_for_every_round():
    """At four times the device's comfortable rate, batches that wait only for
    their own generation round keep the device busier than batches that take
    every admitted request and wait for the latest round (the loop's former
    policy, replayed here as a subclass)."""
    import paper_2108_02025_amd.serve as S

    class LatestRound(S.Scheduler):
        def next_batch(self):
            ids = list(self.ready)[: self.max_batch]
            for _ in ids:
                self.ready.popleft()
            pend = [r for r in self.round_of[ids] if r > self.gen_done]
            return ids, (self.round_token[max(pend)] if pend else None)

    arr, db = _trace(3000, 4e5, 501)
    rates = {}
    for name, cls, kw in (("rounds", S.Scheduler, {}),
                          ("latest", LatestRound, dict(max_round_bytes=1 << 62, max_batch_bytes=1 << 62))):
        orig, S.Scheduler = S.Scheduler, cls
        try:
            sched, ex = run_sim(arr, db, 4 << 30, **kw)
        finally:
            S.Scheduler = orig
        assert (sched.status == 1).all()
        rates[name] = len(arr) / np.nanmax(sched.t_done)
    assert rates["rounds"] > 1.2 * rates["latest"], rates
