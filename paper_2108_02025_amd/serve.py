"""Continuous-batching GEMV server on one MI355X (serving form of the
streaming core).

Requests c = A x (A m x n, binary32 or bfloat16-A with per-row scales, x and
c binary32) arrive on a trace.  The host loop:

  1. releases each request at its arrival time into a FIFO queue;
  2. admits the queue head when its operands fit the HBM budget (a first-fit
     pool carved from one device buffer); admission never skips the head, so
     no request starves;
  3. materialises the operands on the device, on a generation stream: A and
     x from SplitMix64 counters (seeded per request), c zeroed; bfloat16
     requests are quantised per row right away;
  4. whenever fewer than `max_inflight` batches are on the GPU, packs every
     materialised request into the next batch, writes its table and replays
     a captured launch of the batched persistent kernel (one HIP graph per
     table, tables double-buffered so a new batch is written while the
     previous one runs);
  5. polls the batches' completion events, stamps completions and frees
     their memory, which lets queued requests in.

Requests that arrive while others are on the GPU are admitted as memory
frees up and their generation overlaps the running batch.  A request's
result depends only on the request (its configuration comes from its shape
and kind), so it is bit-identical alone and in any mix.

Latency is host-observed completion minus scheduled arrival; aggregate
throughput is the requests' algorithmic bytes over (last completion - first
arrival).
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np
import torch

from . import (SB_BF16, BatchTable, GemvProblem, sb_fill_uniform, sb_gemv_batched, sb_gemv_batched_table_bytes,
               sb_quantize_rows)

ALIGN = 256


@dataclasses.dataclass
class Request:
    id: int
    arrival: float
    kind: str          # "f32" or "bf16"
    m: int
    n: int
    seed: int
    t_admit: float = math.nan
    t_launch: float = math.nan
    t_done: float = math.nan
    batch: int = -1
    offset: int = -1
    problem: GemvProblem | None = None
    result_at: int = -1   # offset of this request's c in the result store (sampled requests)

    @property
    def device_bytes(self) -> int:
        return device_bytes(self.kind, self.m, self.n)

    @property
    def algorithmic_bytes(self) -> int:
        es = 4 if self.kind == "f32" else 2
        return es * self.m * self.n + 4 * self.n + 8 * self.m + (4 * self.m if self.kind == "bf16" else 0)


def _up(v: int) -> int:
    return (v + ALIGN - 1) // ALIGN * ALIGN


def device_bytes(kind: str, m: int, n: int) -> int:
    """Resident bytes of one request: A (or codes + scales), x and c."""
    es = 4 if kind == "f32" else 2
    return _up(es * m * n) + (_up(4 * m) if kind == "bf16" else 0) + _up(4 * n) + _up(4 * m)


def make_trace(n_requests: int = 4096, rate: float = 1e5, seed: int = 501, lo: int = 64, hi: int = 8192,
               bf16_fraction: float = 0.5) -> list[Request]:
    """Poisson arrivals at `rate` requests/s; m and n log-uniform in [lo, hi];
    kind bfloat16-A with probability `bf16_fraction`, else binary32."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    arrivals -= arrivals[0]
    m = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n_requests))).astype(int)
    n = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n_requests))).astype(int)
    kinds = np.where(rng.random(n_requests) < bf16_fraction, "bf16", "f32")
    return [Request(i, float(arrivals[i]), str(kinds[i]), int(m[i]), int(n[i]), seed * (1 << 32) + i)
            for i in range(n_requests)]


class Pool:
    """First-fit allocator over [0, capacity) in ALIGN-byte units (host
    bookkeeping of one device buffer)."""

    def __init__(self, capacity: int):
        self.capacity = capacity
        self.free_list = [(0, capacity)]  # sorted (offset, size)
        self.used = 0

    def alloc(self, nbytes: int) -> int | None:
        nbytes = _up(nbytes)
        for k, (off, size) in enumerate(self.free_list):
            if size >= nbytes:
                if size == nbytes:
                    self.free_list.pop(k)
                else:
                    self.free_list[k] = (off + nbytes, size - nbytes)
                self.used += nbytes
                return off
        return None

    def free(self, off: int, nbytes: int) -> None:
        nbytes = _up(nbytes)
        self.used -= nbytes
        fl = self.free_list
        lo, hi = 0, len(fl)
        while lo < hi:
            mid = (lo + hi) // 2
            if fl[mid][0] < off:
                lo = mid + 1
            else:
                hi = mid
        fl.insert(lo, (off, nbytes))
        # merge with neighbours
        if lo + 1 < len(fl) and fl[lo][0] + fl[lo][1] == fl[lo + 1][0]:
            fl[lo] = (fl[lo][0], fl[lo][1] + fl[lo + 1][1])
            fl.pop(lo + 1)
        if lo > 0 and fl[lo - 1][0] + fl[lo - 1][1] == fl[lo][0]:
            fl[lo - 1] = (fl[lo - 1][0], fl[lo - 1][1] + fl[lo][1])
            fl.pop(lo)


def materialise(buf: torch.Tensor, off: int, kind: str, m: int, n: int, seed: int, stage: torch.Tensor | None,
                config=None) -> GemvProblem:
    """Carve the request's operands out of `buf` at `off` and generate them
    on the current stream.  A uses counters [0, mn), x uses [mn, mn + n);
    c starts at zero.  bfloat16 requests generate A in binary32 into `stage`
    and quantise it per row (as sb_quantize_rows)."""
    cfg = config or {}
    es = 4 if kind == "f32" else 2
    p = off
    a_bytes = es * m * n
    A = buf[p:p + a_bytes]
    p += _up(a_bytes)
    scales = None
    if kind == "bf16":
        scales = buf[p:p + 4 * m].view(torch.float32)
        p += _up(4 * m)
    x = buf[p:p + 4 * n].view(torch.float32)
    p += _up(4 * n)
    c = buf[p:p + 4 * m].view(torch.float32)
    if kind == "f32":
        A = A.view(torch.float32).view(m, n)
        sb_fill_uniform(A.view(-1), seed, 0)
    else:
        A = A.view(torch.int16).view(m, n)
        tmp = stage[: m * n].view(m, n)
        sb_fill_uniform(tmp.view(-1), seed, 0)
        sb_quantize_rows(tmp, A, scales, SB_BF16)
    sb_fill_uniform(x, seed, m * n)
    c.zero_()
    return GemvProblem(A, x, c, scales=scales, q=SB_BF16 if kind == "bf16" else None,
                       group=cfg.get("group", 0), rows_per_tile=cfg.get("rows_per_tile", 0),
                       split=cfg.get("split", 0))


@dataclasses.dataclass
class Stats:
    n: int
    rejected: int
    span_s: float
    achieved_rate: float
    p50_ms: float
    p99_ms: float
    p999_ms: float
    queue_p50_ms: float
    materialise_p50_ms: float
    execute_p50_ms: float
    aggregate_GBs: float
    device_busy_GBs: float
    batches: int
    mean_batch: float
    total_bytes: int

    def as_dict(self) -> dict:
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in dataclasses.asdict(self).items()}


class Server:
    """See the module docstring.  `tuning` maps (kind, m, n) to a
    configuration dict for the batched kernel (or None for automatic)."""

    def __init__(self, budget_bytes: int = 4 << 30, max_batch: int = 512, max_inflight: int = 2,
                 use_graphs: bool = True, tuning=None, sample_every: int = 16, table_bytes: int = 96 << 20,
                 device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.budget = int(budget_bytes)
        self.buf = torch.empty(self.budget, dtype=torch.uint8, device=self.device)
        self.stage = torch.empty(8192 * 8192, dtype=torch.float32, device=self.device)
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.use_graphs = use_graphs
        self.tuning = tuning
        self.sample_every = sample_every
        self.exec_stream = torch.cuda.Stream(device=self.device)
        self.gen_stream = torch.cuda.Stream(device=self.device)
        self.tables = [BatchTable(table_bytes, self.device) for _ in range(max_inflight)]
        self.graphs: list[torch.cuda.CUDAGraph | None] = [None] * max_inflight

    # -- graph of one table's launch ------------------------------------
    def _graph_for(self, k: int) -> torch.cuda.CUDAGraph:
        g = self.graphs[k]
        if g is None:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=self.exec_stream):
                self.tables[k].run()
            self.graphs[k] = g
        return g

    def _config(self, r: Request):
        return self.tuning(r.kind, r.m, r.n) if self.tuning else None

    def warm_up(self, trace: list[Request]) -> None:
        """Capture the graphs with a tiny batch so capture is off the clock."""
        if not self.use_graphs:
            return
        r = Request(-1, 0.0, "f32", 64, 64, 12345)
        with torch.cuda.stream(self.exec_stream):
            P = materialise(self.buf, 0, r.kind, r.m, r.n, r.seed, self.stage)
            for k in range(len(self.tables)):
                self.tables[k].encode([P])
                self.tables[k].run()  # eager launch before capture
            torch.cuda.synchronize()
            for k in range(len(self.tables)):
                self._graph_for(k)
        torch.cuda.synchronize()

    def run(self, trace: list[Request]) -> Stats:
        n_req = len(trace)
        pool = Pool(self.budget)
        sampled = [r for r in trace if r.id % self.sample_every == 0]
        self.results = torch.empty(max(1, sum(r.m for r in sampled)), dtype=torch.float32, device=self.device)
        pos = 0
        for r in sampled:
            r.result_at = pos
            pos += r.m
        queue: collections.deque[Request] = collections.deque()
        ready: list[Request] = []
        inflight: collections.deque = collections.deque()
        free_tables = collections.deque(range(len(self.tables)))
        gen_event = None
        done = rejected = 0
        nxt = 0
        batch_id = 0
        busy_events = []
        self.warm_up(trace)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while done + rejected < n_req:
            now = time.perf_counter() - t0
            while nxt < n_req and trace[nxt].arrival <= now:
                queue.append(trace[nxt])
                nxt += 1
            # admission: FIFO, by device memory
            while queue:
                r = queue[0]
                if r.device_bytes > self.budget:
                    queue.popleft()
                    rejected += 1
                    r.t_done = math.inf
                    continue
                off = pool.alloc(r.device_bytes)
                if off is None:
                    break
                queue.popleft()
                r.offset = off
                r.t_admit = time.perf_counter() - t0
                with torch.cuda.stream(self.gen_stream):
                    r.problem = materialise(self.buf, off, r.kind, r.m, r.n, r.seed, self.stage, self._config(r))
                    gen_event = torch.cuda.Event()
                    gen_event.record()
                ready.append(r)
            # continuous batching: launch whatever is ready when a table is free
            if ready and free_tables:
                k = free_tables.popleft()
                batch, ready = ready[: self.max_batch], ready[self.max_batch:]
                with torch.cuda.stream(self.exec_stream):
                    self.exec_stream.wait_event(gen_event)
                    start = torch.cuda.Event(enable_timing=True)
                    end = torch.cuda.Event(enable_timing=True)
                    self.tables[k].encode([r.problem for r in batch])
                    start.record()
                    if self.use_graphs:
                        self._graph_for(k).replay()
                    else:
                        self.tables[k].run()
                    end.record()
                    for r in batch:
                        if r.result_at >= 0:
                            self.results[r.result_at:r.result_at + r.m].copy_(r.problem.c)
                    fin = torch.cuda.Event()
                    fin.record()
                t = time.perf_counter() - t0
                for r in batch:
                    r.t_launch = t
                    r.batch = batch_id
                inflight.append((fin, batch, k, start, end))
                busy_events.append((start, end))
                batch_id += 1
            # completions
            while inflight and inflight[0][0].query():
                fin, batch, k, _, _ = inflight.popleft()
                t = time.perf_counter() - t0
                for r in batch:
                    r.t_done = t
                    pool.free(r.offset, r.device_bytes)
                    r.problem = None
                done += len(batch)
                free_tables.append(k)
        torch.cuda.synchronize()
        return self._stats(trace, busy_events, batch_id, rejected)

    def _stats(self, trace, busy_events, nbatches, rejected) -> Stats:
        ok = [r for r in trace if math.isfinite(r.t_done)]
        lat = np.array([r.t_done - r.arrival for r in ok])
        q = np.array([r.t_admit - r.arrival for r in ok])
        mat = np.array([r.t_launch - r.t_admit for r in ok])
        ex = np.array([r.t_done - r.t_launch for r in ok])
        total = sum(r.algorithmic_bytes for r in ok)
        span = max(r.t_done for r in ok) - min(r.arrival for r in ok)
        busy = sum(a.elapsed_time(b) for a, b in busy_events) * 1e-3
        pct = lambda a, p: float(np.percentile(a, p)) * 1e3  # noqa: E731
        return Stats(
            n=len(ok), rejected=rejected, span_s=span, achieved_rate=len(ok) / span,
            p50_ms=pct(lat, 50), p99_ms=pct(lat, 99), p999_ms=pct(lat, 99.9),
            queue_p50_ms=pct(q, 50), materialise_p50_ms=pct(mat, 50), execute_p50_ms=pct(ex, 50),
            aggregate_GBs=total / span / 1e9, device_busy_GBs=total / busy / 1e9 if busy > 0 else math.nan,
            batches=nbatches, mean_batch=len(ok) / max(nbatches, 1), total_bytes=total)

    def result_of(self, r: Request) -> torch.Tensor:
        return self.results[r.result_at:r.result_at + r.m]

    def rerun_alone(self, r: Request) -> torch.Tensor:
        """Regenerate one request's operands and run it alone (same
        configuration); returns its output."""
        buf = torch.empty(r.device_bytes, dtype=torch.uint8, device=self.device)
        P = materialise(buf, 0, r.kind, r.m, r.n, r.seed, self.stage, self._config(r))
        sb_gemv_batched([P])
        torch.cuda.synchronize()
        return P.c.clone()
