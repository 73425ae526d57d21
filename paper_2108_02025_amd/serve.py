"""Continuous-batching GEMV server on one MI355X (serving form of the
streaming core).

Requests c = A x (A m x n, binary32 or bfloat16-A with per-row scales, x and
c binary32) and DOT requests alpha = x . y (binary32; served as the one-row
GEMV whose row is x, which is the same sum) arrive on a trace.  The host
loop (Scheduler, driven here by GpuExecutor and the wall clock):

  1. releases each request at its arrival time into a FIFO queue, and drops
     queued requests that were cancelled or whose admission deadline passed;
  2. admits the queue head while its operands fit the HBM budget (a
     first-fit pool carved from one device buffer) and the admission round
     stays under a byte cap; admission never skips the head, so no request
     starves;
  3. materialises the operands of every request admitted in a round with
     one launch of the batched generator on a generation stream: A and x
     from SplitMix64 counters (seeded per request), c zeroed, bfloat16 rows
     scaled and encoded in the same kernel;
  4. whenever one of `max_inflight` tables is free, packs the admitted
     requests into the next batch (at most one generation round still
     running, under a byte cap), writes its table and replays a captured
     launch of the batched persistent kernel (one HIP graph per table) on
     the execution stream, behind that round's generation event;
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
import ctypes
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
    op: str = "gemv"   # "dot": alpha = x . y, the one-row binary32 GEMV (m = 1)
    deadline: float = math.inf   # trace time by which it must be admitted, else it expires unserved
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
               bf16_fraction: float = 0.5, dot_fraction: float = 0.0, dot_hi: int | None = None) -> list[Request]:
    """Poisson arrivals at `rate` requests/s; m and n log-uniform in [lo, hi];
    kind bfloat16-A with probability `bf16_fraction`, else binary32.  With
    `dot_fraction` > 0 that share of requests are binary32 DOTs of length
    log-uniform in [lo, dot_hi] (default hi), drawn after the GEMV fields so
    the rest of the trace does not change."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    arrivals -= arrivals[0]
    m = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n_requests))).astype(int)
    n = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n_requests))).astype(int)
    kinds = np.where(rng.random(n_requests) < bf16_fraction, "bf16", "f32")
    ops = np.full(n_requests, "gemv")
    if dot_fraction > 0:
        is_dot = rng.random(n_requests) < dot_fraction
        dn = np.rint(np.exp(rng.uniform(math.log(lo), math.log(dot_hi or hi), n_requests))).astype(int)
        ops[is_dot], kinds[is_dot], m[is_dot], n[is_dot] = "dot", "f32", 1, dn[is_dot]
    return [Request(i, float(arrivals[i]), str(kinds[i]), int(m[i]), int(n[i]), seed * (1 << 32) + i, str(ops[i]))
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
    dot_requests: int = 0

    def as_dict(self) -> dict:
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in dataclasses.asdict(self).items()}


GEMV_DESC = np.dtype([("dtype", "<i4"), ("group", "<i4"), ("rows_per_tile", "<i4"), ("split", "<i4"),
                      ("m", "<i8"), ("n", "<i8"), ("lda", "<i8"),
                      ("A", "<u8"), ("scales", "<u8"), ("x", "<u8"), ("c", "<u8"),
                      ("layout", "<i4"), ("op", "<i4")])
GEN_DESC = np.dtype([("dtype", "<i4"), ("reserved", "<i4"), ("m", "<i8"), ("n", "<i8"), ("lda", "<i8"),
                     ("seed", "<u8"), ("A", "<u8"), ("scales", "<u8"), ("x", "<u8"), ("c", "<u8")])
assert GEMV_DESC.itemsize == 80 and GEN_DESC.itemsize == 72


# ------------------------------------------------------------------ policy --

class Scheduler:
    """The serving loop's host policy, independent of the device.  It sees
    the device through an executor (generate / launch / finished) and time
    through a clock (now / idle), so the same code drives the GPU and a
    simulated device in tests.

    Per turn of the loop:
      1. requests whose arrival time has passed join a FIFO queue; queued
         requests whose deadline has passed, or that were cancelled, leave
         it unserved;
      2. admission: the queue head is admitted while its device bytes fit
         the pool and the round's byte cap; a request larger than the whole
         budget is rejected; the head is never skipped, so no request
         starves behind smaller ones.  The round's operands are generated by
         one executor call;
      3. batching: while a table is free, the admitted requests go into the
         next batch in admission order, up to max_batch requests and
         max_batch_bytes.  A batch takes the requests whose generation has
         finished and, after them, those of the next generation round still
         running (its launch waits for that round on the device), never a
         later round: a batch never waits for generation admitted after its
         requests, so a backlog drains with generation and execution
         overlapped instead of each batch waiting for the newest round;
      4. finished batches free their requests' memory and their table.
    Requests are completed in batch order; each request's result depends
    only on the request.
    """

    def __init__(self, dev_bytes: np.ndarray, budget: int, max_batch: int = 512, max_inflight: int = 2,
                 max_round_bytes: int = 256 << 20, max_batch_bytes: int = 512 << 20):
        self.dev_bytes = np.asarray(dev_bytes, dtype=np.int64)
        N = len(self.dev_bytes)
        self.budget = int(budget)
        self.max_batch = max_batch
        self.max_round_bytes = int(max_round_bytes)
        self.max_batch_bytes = int(max_batch_bytes)
        self.pool = Pool(self.budget)
        self.queue: collections.deque[int] = collections.deque()
        self.ready: collections.deque[int] = collections.deque()   # admitted, not yet in a batch
        self.rounds: collections.deque = collections.deque()       # (round id, token) still generating
        self.round_token: dict[int, object] = {}
        self.round_of = np.full(N, -1, dtype=np.int64)
        self.gen_done = -1                                          # every round <= this has finished
        self.n_rounds = 0
        self.inflight: collections.deque = collections.deque()     # (token, ids, table)
        self.free_tables = collections.deque(range(max_inflight))
        self.offset = np.full(N, -1, dtype=np.int64)
        self.t_admit = np.full(N, np.nan)
        self.t_launch = np.full(N, np.nan)
        self.t_done = np.full(N, np.nan)
        self.deadline = np.full(N, np.inf)
        self.cancelled = np.zeros(N, dtype=bool)
        self.status = np.zeros(N, dtype=np.int8)   # 0 pending, 1 done, 2 rejected, 3 expired or cancelled
        self.finished = 0
        self.batches = 0
        self.max_queue = 0
        self._cancel_pending = False
        self._deadlines = False

    # -- requests leaving the queue unserved --------------------------------
    def cancel(self, i: int) -> bool:
        """Cancel request i if it has not been admitted yet (it then leaves
        the queue unserved); returns whether it was."""
        if self.status[i] != 0 or self.offset[i] >= 0:
            return False
        self.cancelled[i] = True
        self._cancel_pending = True
        return True

    def _drop(self, i: int, status: int) -> None:
        self.status[i] = status
        self.t_done[i] = np.inf
        self.finished += 1

    def _expire(self, now: float) -> bool:
        if not self.queue or not (self._cancel_pending or self._deadlines):
            return False
        self._cancel_pending = False
        q = self.queue
        gone = [i for i in q if self.cancelled[i] or self.deadline[i] < now]
        if not gone:
            return False
        keep = set(gone)
        self.queue = collections.deque(i for i in q if i not in keep)
        for i in gone:
            self._drop(i, 3)
        return True

    # -- admission ------------------------------------------------------------
    def admit(self, now: float) -> list[int]:
        admitted, nbytes = [], 0
        while self.queue:
            i = self.queue[0]
            b = int(self.dev_bytes[i])
            if b > self.budget:
                self.queue.popleft()
                self._drop(i, 2)
                continue
            if admitted and nbytes + b > self.max_round_bytes:
                break
            off = self.pool.alloc(b)
            if off is None:
                break
            self.queue.popleft()
            self.offset[i] = off
            admitted.append(i)
            nbytes += b
        if admitted:
            self.t_admit[admitted] = now
        return admitted

    # -- batching -------------------------------------------------------------
    def next_batch(self) -> tuple[list[int], object]:
        """Ids of the next batch and the generation token its launch must wait
        for (None when every request in it has been generated)."""
        ids, nbytes, wait_round = [], 0, None
        for i in self.ready:
            r = int(self.round_of[i])
            if r > self.gen_done:
                if wait_round is None:
                    wait_round = r
                elif r != wait_round:
                    break
            b = int(self.dev_bytes[i])
            if ids and (len(ids) >= self.max_batch or nbytes + b > self.max_batch_bytes):
                break
            ids.append(i)
            nbytes += b
        for _ in ids:
            self.ready.popleft()
        return ids, (self.round_token[wait_round] if wait_round is not None else None)

    # -- the loop -------------------------------------------------------------
    def serve(self, arrival: np.ndarray, executor, clock) -> None:
        N = len(arrival)
        nxt = 0
        self._deadlines = bool(np.isfinite(self.deadline).any())
        while self.finished < N:
            busy = False
            now = clock.now()
            upto = int(np.searchsorted(arrival, now, side="right"))
            if upto > nxt:
                self.queue.extend(range(nxt, upto))
                nxt = upto
                self.max_queue = max(self.max_queue, len(self.queue))
            busy |= self._expire(now)
            ids = self.admit(now)
            if ids:
                busy = True
                tok = executor.generate(np.array(ids), self.offset)
                self.round_of[ids] = self.n_rounds
                self.rounds.append((self.n_rounds, tok))
                self.round_token[self.n_rounds] = tok
                self.ready.extend(ids)
                self.n_rounds += 1
            while self.rounds and executor.finished(self.rounds[0][1]):
                self.gen_done = self.rounds.popleft()[0]
                del self.round_token[self.gen_done]
            while self.free_tables and self.ready:
                batch, wait = self.next_batch()
                if not batch:
                    break
                busy = True
                k = self.free_tables.popleft()
                b = np.array(batch)
                tok = executor.launch(b, self.offset, k, wait)
                self.t_launch[b] = clock.now()
                self.inflight.append((tok, b, k))
                self.batches += 1
            while self.inflight and executor.finished(self.inflight[0][0]):
                tok, b, k = self.inflight.popleft()
                self.t_done[b] = clock.now()
                self.status[b] = 1
                for i in b:
                    self.pool.free(int(self.offset[i]), int(self.dev_bytes[i]))
                self.finished += len(b)
                self.free_tables.append(k)
                busy = True
            if not busy:
                clock.idle(arrival[nxt] if nxt < N else np.inf, executor)


class WallClock:
    """Seconds since the first call; idle() spins (the loop polls)."""

    def __init__(self):
        self.t0 = None

    def now(self) -> float:
        if self.t0 is None:
            self.t0 = time.perf_counter()
        return time.perf_counter() - self.t0

    def idle(self, next_arrival: float, executor) -> None:
        return None


# ----------------------------------------------------------------- device --

class GpuExecutor:
    """The device side of the serving loop: operand generation on the
    generation stream, batched launches (captured graphs over
    double-buffered tables) on the execution stream, completion through
    events."""

    def __init__(self, server: "Server", desc_all: np.ndarray, gen_all: np.ndarray, rel: np.ndarray,
                 has_s: np.ndarray, result_at: np.ndarray, c_rel: np.ndarray, m: np.ndarray):
        self.s = server
        self.desc_all, self.gen_all, self.rel, self.has_s = desc_all, gen_all, rel, has_s
        self.result_at, self.c_rel, self.m = result_at, c_rel, m
        self.busy_events = []

    def _addresses(self, table, ids, offset):
        base = (self.s.base + offset[ids]).astype(np.uint64)
        table["A"] = base
        table["scales"] = (base + self.rel[ids, 1]) * self.has_s[ids]
        table["x"] = base + self.rel[ids, 2]
        table["c"] = base + self.rel[ids, 3]
        return table

    def generate(self, ids, offset):
        self.s._generate(self._addresses(self.gen_all[ids], ids, offset))
        ev = torch.cuda.Event()
        ev.record(self.s.gen_stream)
        return ev

    def launch(self, ids, offset, k, wait):
        s = self.s
        d = self._addresses(self.desc_all[ids], ids, offset)
        with torch.cuda.stream(s.exec_stream):
            if wait is not None:
                s.exec_stream.wait_event(wait)
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            s.tables[k].encode_descs(d.ctypes.data, len(ids))
            start.record()
            if s.use_graphs:
                s._graph_for(k).replay()
            else:
                s.tables[k].run()
            end.record()
            for i in ids[self.result_at[ids] >= 0]:
                c_off = int(offset[i] + self.c_rel[i])
                s.results[self.result_at[i]:self.result_at[i] + self.m[i]].copy_(
                    s.buf[c_off:c_off + 4 * int(self.m[i])].view(torch.float32))
            fin = torch.cuda.Event()
            fin.record()
        self.busy_events.append((start, end))
        return fin

    def finished(self, ev) -> bool:
        return ev.query()


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
    dot_requests: int = 0
    expired: int = 0
    rounds: int = 0
    max_queue: int = 0
    trace_rate: float = math.nan    # the trace's own arrival rate, (N - 1) / (last - first arrival)

    def as_dict(self) -> dict:
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in dataclasses.asdict(self).items()}


_STREAMS: dict[int, tuple[torch.cuda.Stream, torch.cuda.Stream]] = {}


def serving_streams(device: torch.device) -> tuple[torch.cuda.Stream, torch.cuda.Stream]:
    """The execution and generation streams of a device, created once per
    process and shared by every Server on it.  HIP spreads streams over a few
    hardware queues in creation order; a fresh pair per Server could land on
    one queue, where the generation launches and the batched launches would
    run one after another instead of side by side."""
    idx = device.index or 0
    if idx not in _STREAMS:
        _STREAMS[idx] = (torch.cuda.Stream(device=device), torch.cuda.Stream(device=device))
    return _STREAMS[idx]


class Server:
    """Continuous-batching GEMV server on one GPU (see the module docstring
    and Scheduler).  `tuning` maps (kind, m, n) to a configuration dict for
    the batched kernel (or None for automatic).  `executor_class` is the
    device side of the loop (GpuExecutor)."""

    executor_class = GpuExecutor

    def __init__(self, budget_bytes: int = 4 << 30, max_batch: int = 512, max_inflight: int = 2,
                 use_graphs: bool = True, tuning=None, sample_every: int = 16, table_bytes: int = 96 << 20,
                 device=None, max_round_bytes: int = 256 << 20, max_batch_bytes: int = 512 << 20):
        from . import Handle
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.budget = int(budget_bytes)
        self.buf = torch.empty(self.budget, dtype=torch.uint8, device=self.device)
        self.base = self.buf.data_ptr()
        self.stage = torch.empty(8192 * 8192, dtype=torch.float32, device=self.device)
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.max_round_bytes = max_round_bytes
        self.max_batch_bytes = max_batch_bytes
        self.use_graphs = use_graphs
        self.tuning = tuning
        self.sample_every = sample_every
        self.exec_stream, self.gen_stream = serving_streams(self.device)
        self.gen_handle = Handle(self.device.index)
        with torch.cuda.stream(self.gen_stream):
            self.gen_handle.prepare(1 << 16)  # bound to the generation stream from here on
        self.tables = [BatchTable(table_bytes, self.device) for _ in range(max_inflight)]
        self.graphs: list[torch.cuda.CUDAGraph | None] = [None] * max_inflight
        self.scheduler: Scheduler | None = None

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

    def warm_up(self) -> None:
        """Run every kernel of the loop once (the operand generator on a
        binary32 and a bfloat16 request, the batched launch), capture the
        graphs and replay them, so first-use costs stay off the clock."""
        gen = np.zeros(2, dtype=GEN_DESC)
        per = device_bytes("bf16", 64, 64)
        for k, (dt, kind) in enumerate(((1, "f32"), (2, "bf16"))):
            base = self.base + k * per
            es = 4 if kind == "f32" else 2
            a = _up(es * 64 * 64)
            s = _up(4 * 64) if kind == "bf16" else 0
            gen[k] = (dt, 0, 64, 64, 64, 1 + k, base, base + a if s else 0, base + a + s, base + a + s + _up(4 * 64))
        with torch.cuda.stream(self.gen_stream):
            self._generate(gen)
        torch.cuda.synchronize()
        if not self.use_graphs:
            return
        with torch.cuda.stream(self.exec_stream):
            P = materialise(self.buf, 0, "f32", 64, 64, 12345, self.stage)
            for k in range(len(self.tables)):
                self.tables[k].encode([P])
                self.tables[k].run()  # eager launch before capture
            torch.cuda.synchronize()
            for k in range(len(self.tables)):
                self._graph_for(k)
            torch.cuda.synchronize()
            # replay each graph a few times: the first launches of an
            # instantiated graph cost far more than later ones
            for _ in range(3):
                for k in range(len(self.tables)):
                    self.graphs[k].replay()
                torch.cuda.synchronize()
        torch.cuda.synchronize()

    def _generate(self, gen: np.ndarray) -> None:
        """One sb_generate_batched launch on the generation stream."""
        from . import load
        L = load()
        h = self.gen_handle
        need = int(L.sb_generate_batched_bytes(len(gen)))
        if h._ws is None or h._ws.numel() < need:
            with torch.cuda.stream(self.gen_stream):
                h.prepare(max(need, 1 << 16))
        h.check(L.sb_generate_batched(h.h, ctypes.c_void_p(gen.ctypes.data), len(gen)))

    def run(self, trace: list[Request], warm_requests: int = 512) -> Stats:
        """Serve `trace` and return its statistics.  Before the clock starts,
        warm_up() runs every kernel once and a short untimed trace of
        `warm_requests` requests (other seeds, the measured trace's shape
        range, the same rate) goes through the same loop: the first turns of
        a fresh loop pay one-off costs (lazily loaded runtime kernels, first
        launches of the graphs, workspace growth, the first touch of the
        pool's pages) that otherwise start the measured trace with a
        backlog."""
        self.warm_up()
        if warm_requests > 0 and trace:
            lo = min(min(r.m, r.n) for r in trace if r.op == "gemv") if any(r.op == "gemv" for r in trace) else 64
            hi = max(max(r.m, r.n) for r in trace if r.op == "gemv") if any(r.op == "gemv" for r in trace) else 64
            span = trace[-1].arrival - trace[0].arrival
            rate = (len(trace) - 1) / span if span > 0 else 1e5
            warm = make_trace(warm_requests, rate=rate, seed=0x5EED, lo=lo, hi=hi, dot_fraction=0.25)
            self._serve(warm, warm=True)
        return self._serve(trace)

    def _serve(self, trace: list[Request], warm: bool = False) -> Stats | None:
        N = len(trace)
        arrival = np.array([r.arrival for r in trace])
        m = np.array([r.m for r in trace], dtype=np.int64)
        n = np.array([r.n for r in trace], dtype=np.int64)
        bf16 = np.array([r.kind == "bf16" for r in trace])
        seed = np.array([r.seed for r in trace], dtype=np.uint64)
        es = np.where(bf16, 2, 4)
        a_bytes = (es * m * n + ALIGN - 1) // ALIGN * ALIGN
        s_bytes = np.where(bf16, (4 * m + ALIGN - 1) // ALIGN * ALIGN, 0)
        x_bytes = (4 * n + ALIGN - 1) // ALIGN * ALIGN
        dev_bytes = a_bytes + s_bytes + x_bytes + (4 * m + ALIGN - 1) // ALIGN * ALIGN
        cfg = np.zeros((N, 3), dtype=np.int32)
        if self.tuning:
            for i, r in enumerate(trace):
                c = self.tuning(r.kind, r.m, r.n) or {}
                cfg[i] = (c.get("group", 0), c.get("rows_per_tile", 0), c.get("split", 0))
        # Every request's generation and GEMV descriptors, built once with
        # addresses relative to its operand block; a turn of the loop gathers
        # the rows it needs and adds the blocks' device addresses.
        rel = np.zeros((N, 4), dtype=np.uint64)  # A, scales, x, c
        rel[:, 1] = np.where(bf16, a_bytes, 0)
        rel[:, 2] = a_bytes + s_bytes
        rel[:, 3] = a_bytes + s_bytes + x_bytes
        has_s = bf16.astype(np.uint64)
        gen_all = np.zeros(N, dtype=GEN_DESC)
        gen_all["dtype"] = np.where(bf16, 2, 1)
        gen_all["m"], gen_all["n"], gen_all["lda"], gen_all["seed"] = m, n, n, seed
        desc_all = np.zeros(N, dtype=GEMV_DESC)
        desc_all["dtype"] = np.where(bf16, 2, 1)
        desc_all["group"], desc_all["rows_per_tile"], desc_all["split"] = cfg[:, 0], cfg[:, 1], cfg[:, 2]
        desc_all["m"], desc_all["n"], desc_all["lda"] = m, n, n

        sampled = np.flatnonzero(np.arange(N) % self.sample_every == 0)
        result_at = np.full(N, -1, dtype=np.int64)
        result_at[sampled] = np.concatenate([[0], np.cumsum(m[sampled])[:-1]]) if len(sampled) else []
        self.results = torch.empty(max(1, int(m[sampled].sum())), dtype=torch.float32, device=self.device)

        sched = Scheduler(dev_bytes, self.budget, self.max_batch, self.max_inflight, self.max_round_bytes,
                          self.max_batch_bytes)
        sched.deadline[:] = [r.deadline for r in trace]
        ex = self.executor_class(self, desc_all, gen_all, rel, has_s, result_at, rel[:, 3].astype(np.int64), m)
        torch.cuda.synchronize()
        sched.serve(arrival, ex, WallClock())
        torch.cuda.synchronize()
        if warm:
            return None
        self.scheduler = sched
        for i, r in enumerate(trace):
            r.t_admit, r.t_launch, r.t_done = float(sched.t_admit[i]), float(sched.t_launch[i]), float(sched.t_done[i])
            r.offset, r.result_at = int(sched.offset[i]), int(result_at[i])
        return stats_of(trace, sched, ex.busy_events)


    def result_of(self, r: Request) -> torch.Tensor:
        return self.results[r.result_at:r.result_at + r.m]

    def rerun_alone(self, r: Request) -> torch.Tensor:
        """Regenerate one request's operands with the separate fill and
        quantise calls and run it alone (same configuration); returns its
        output."""
        buf = torch.empty(r.device_bytes, dtype=torch.uint8, device=self.device)
        P = materialise(buf, 0, r.kind, r.m, r.n, r.seed, self.stage, self._config(r))
        sb_gemv_batched([P])
        torch.cuda.synchronize()
        return P.c.clone()


def stats_of(trace: list[Request], sched: Scheduler, busy_events=()) -> Stats:
    """Latency and throughput of a served trace (completion minus scheduled
    arrival; aggregate bytes over last completion minus first arrival)."""
    ok = [r for r in trace if math.isfinite(r.t_done)]
    lat = np.array([r.t_done - r.arrival for r in ok])
    q = np.array([r.t_admit - r.arrival for r in ok])
    mat = np.array([r.t_launch - r.t_admit for r in ok])
    ex = np.array([r.t_done - r.t_launch for r in ok])
    total = sum(r.algorithmic_bytes for r in ok)
    span = max(r.t_done for r in ok) - min(r.arrival for r in ok) if ok else math.nan
    busy = sum(a.elapsed_time(b) for a, b in busy_events) * 1e-3
    pct = (lambda a, p: float(np.percentile(a, p)) * 1e3 if len(a) else math.nan)  # noqa: E731
    return Stats(
        n=len(ok), rejected=int((sched.status == 2).sum()), span_s=span,
        achieved_rate=len(ok) / span if ok and span > 0 else math.nan,
        p50_ms=pct(lat, 50), p99_ms=pct(lat, 99), p999_ms=pct(lat, 99.9),
        queue_p50_ms=pct(q, 50), materialise_p50_ms=pct(mat, 50), execute_p50_ms=pct(ex, 50),
        aggregate_GBs=total / span / 1e9 if ok and span > 0 else math.nan,
        device_busy_GBs=total / busy / 1e9 if busy > 0 else math.nan,
        batches=sched.batches, mean_batch=len(ok) / max(sched.batches, 1), total_bytes=total,
        dot_requests=sum(r.op == "dot" for r in ok), expired=int((sched.status == 3).sum()),
        rounds=sched.n_rounds, max_queue=sched.max_queue,
        trace_rate=(len(trace) - 1) / (trace[-1].arrival - trace[0].arrival)
        if len(trace) > 1 and trace[-1].arrival > trace[0].arrival else math.nan)

