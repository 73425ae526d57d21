"""Test-only stand-ins for the serving loop's device and clock: a simulated
clock and a model of the GPU with a generation stream and an execution
stream, each running its work in order, with costs charged from a request's
bytes.  The scheduler under test is the library's; only the device is
modelled.  The model also checks what the device would need to be correct:
a batch never starts before its requests' operands are generated, and the
operand blocks alive at any time fit the budget without overlapping."""
from __future__ import annotations

import math

import numpy as np


class SimClock:
    """Simulated seconds.  Host work advances it through spend(); an idle
    loop turn jumps to the next arrival or device event."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def spend(self, dt: float) -> None:
        self.t += dt

    def idle(self, next_arrival: float, executor) -> None:
        nxt = min(next_arrival, executor.next_event(self.t))
        if not math.isfinite(nxt):
            raise AssertionError("the loop is idle with nothing left to wait for")
        self.t = max(self.t + 1e-7, nxt)


class SimExecutor:
    """Device model.  Generation of a round costs gen_fixed + bytes/gen_rate
    on the generation stream; a batch costs exec_fixed + bytes/exec_rate on
    the execution stream and starts no earlier than the generation token it
    was launched with.  Host costs are charged to the clock per call."""

    def __init__(self, clock: SimClock, dev_bytes, budget: int, gen_rate=2.0e12, exec_rate=3.0e12,
                 gen_fixed=4e-6, exec_fixed=8e-6, host_generate=20e-6, host_launch=40e-6, host_poll=1e-6):
        self.clock = clock
        self.dev_bytes = np.asarray(dev_bytes, dtype=np.int64)
        self.budget = budget
        self.gen_rate, self.exec_rate = gen_rate, exec_rate
        self.gen_fixed, self.exec_fixed = gen_fixed, exec_fixed
        self.host_generate, self.host_launch, self.host_poll = host_generate, host_launch, host_poll
        self.gen_free = 0.0
        self.exec_free = 0.0
        self.gen_end = np.full(len(self.dev_bytes), np.nan)
        self.live: dict[int, tuple[int, int]] = {}      # request -> (offset, bytes)
        self.pending: list[float] = []                  # device event times not yet observed
        self.batches: list[tuple[float, float, list[int]]] = []
        self.observed: set = set()
        self.n_tokens = 0

    # executor interface used by the library's Scheduler
    def generate(self, ids, offset):
        self.clock.spend(self.host_generate)
        for i in ids:
            o, b = int(offset[i]), int(self.dev_bytes[i])
            assert o >= 0 and o + b <= self.budget, (i, o, b)
            for j, (oj, bj) in self.live.items():
                assert o + b <= oj or oj + bj <= o, f"request {i} overlaps live request {j}"
            self.live[int(i)] = (o, b)
        start = max(self.clock.now(), self.gen_free)
        end = start + self.gen_fixed + float(self.dev_bytes[ids].sum()) / self.gen_rate
        self.gen_free = end
        self.gen_end[ids] = end
        self.pending.append(end)
        self.n_tokens += 1
        return ("gen", end, tuple(int(i) for i in ids), self.n_tokens)

    def launch(self, ids, offset, table, wait):
        self.clock.spend(self.host_launch)
        assert all(int(i) in self.live for i in ids)
        start = max(self.clock.now(), self.exec_free, wait[1] if wait is not None else 0.0)
        late = [int(i) for i in ids if self.gen_end[i] > start]
        assert not late, f"batch starts at {start} before requests {late} are generated"
        end = start + self.exec_fixed + float(self.dev_bytes[ids].sum()) / self.exec_rate
        self.exec_free = end
        self.pending.append(end)
        self.n_tokens += 1
        tok = ("exec", end, tuple(int(i) for i in ids), self.n_tokens)
        self.batches.append((start, end, list(tok[2])))
        return tok

    def finished(self, tok) -> bool:
        self.clock.spend(self.host_poll)
        done = self.clock.now() >= tok[1]
        if done and tok[0] == "exec" and tok[3] not in self.observed:
            self.observed.add(tok[3])
            for i in tok[2]:
                del self.live[i]
        return done

    def next_event(self, t: float) -> float:
        later = [e for e in self.pending if e > t]
        self.pending = later
        return min(later) if later else math.inf


def run_sim(trace_arrival, dev_bytes, budget, deadlines=None, cancel_at=None, **kw):
    """Serve a trace with the library's Scheduler on the modelled device.
    Returns (scheduler, executor).  cancel_at: {time: [request ids]} cancels
    those requests at the first turn at or after that time."""
    from paper_2108_02025_amd.serve import Scheduler
    sched_kw = {k: kw.pop(k) for k in ("max_batch", "max_inflight", "max_round_bytes", "max_batch_bytes")
                if k in kw}
    clock = SimClock()
    ex = SimExecutor(clock, dev_bytes, budget, **kw)
    sched = Scheduler(dev_bytes, budget, **sched_kw)
    if deadlines is not None:
        sched.deadline[:] = deadlines
    if cancel_at:
        pending = sorted(cancel_at.items())
        base_now = clock.now

        def now():
            t = base_now()
            while pending and pending[0][0] <= t:
                for i in pending.pop(0)[1]:
                    sched.cancel(i)
            return t
        clock.now = now
    sched.serve(np.asarray(trace_arrival, dtype=float), ex, clock)
    return sched, ex
