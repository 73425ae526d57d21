"""Continuous-batching GEMV server on one MI355X (serving form of the
streaming core).

Requests c = A x (A m x n, binary32 or bfloat16-A with per-row scales, x and
c binary32) and DOT requests alpha = x . y (binary32; served as the one-row
GEMV whose row is x, which is the same sum) arrive on a trace.  The host
loop:

  1. releases each request at its arrival time into a FIFO queue;
  2. admits the queue head when its operands fit the HBM budget (a first-fit
     pool carved from one device buffer); admission never skips the head, so
     no request starves;
  3. materialises the operands of every request admitted in a round with
     one launch of the batched generator on a generation stream: A and x
     from SplitMix64 counters (seeded per request), c zeroed, bfloat16 rows
     scaled and encoded in the same kernel;
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
                      ("A", "<u8"), ("scales", "<u8"), ("x", "<u8"), ("c", "<u8")])
GEN_DESC = np.dtype([("dtype", "<i4"), ("reserved", "<i4"), ("m", "<i8"), ("n", "<i8"), ("lda", "<i8"),
                     ("seed", "<u8"), ("A", "<u8"), ("scales", "<u8"), ("x", "<u8"), ("c", "<u8")])
assert GEMV_DESC.itemsize == 72 and GEN_DESC.itemsize == 72


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
    """See the module docstring.  `tuning` maps (kind, m, n) to a
    configuration dict for the batched kernel (or None for automatic)."""

    def __init__(self, budget_bytes: int = 4 << 30, max_batch: int = 512, max_inflight: int = 2,
                 use_graphs: bool = True, tuning=None, sample_every: int = 16, table_bytes: int = 96 << 20,
                 device=None):
        from . import Handle
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.budget = int(budget_bytes)
        self.buf = torch.empty(self.budget, dtype=torch.uint8, device=self.device)
        self.base = self.buf.data_ptr()
        self.stage = torch.empty(8192 * 8192, dtype=torch.float32, device=self.device)
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.use_graphs = use_graphs
        self.tuning = tuning
        self.sample_every = sample_every
        self.exec_stream, self.gen_stream = serving_streams(self.device)
        self.gen_handle = Handle(self.device.index)
        with torch.cuda.stream(self.gen_stream):
            self.gen_handle.prepare(1 << 16)  # bound to the generation stream from here on
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
        `warm_requests` requests (other seeds) goes through the same loop:
        the first turns of a fresh loop pay one-off costs (lazily loaded
        runtime kernels, first launches of the graphs, workspace growth)
        that otherwise start the measured trace with a backlog."""
        self.warm_up()
        if warm_requests > 0:
            warm = make_trace(warm_requests, rate=1e5, seed=0x5EED, hi=4096, dot_fraction=0.25)
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

        def addresses(table, ids):
            base = (self.base + offset[ids]).astype(np.uint64)
            table["A"] = base
            table["scales"] = (base + rel[ids, 1]) * has_s[ids]
            table["x"] = base + rel[ids, 2]
            table["c"] = base + rel[ids, 3]
            return table

        offset = np.full(N, -1, dtype=np.int64)
        t_admit = np.full(N, np.nan)
        t_launch = np.full(N, np.nan)
        t_done = np.full(N, np.nan)
        sampled = np.flatnonzero(np.arange(N) % self.sample_every == 0)
        result_at = np.full(N, -1, dtype=np.int64)
        result_at[sampled] = np.concatenate([[0], np.cumsum(m[sampled])[:-1]]) if len(sampled) else []
        self.results = torch.empty(max(1, int(m[sampled].sum())), dtype=torch.float32, device=self.device)

        pool = Pool(self.budget)
        queue: collections.deque[int] = collections.deque()
        ready: list[int] = []
        inflight: collections.deque = collections.deque()
        free_tables = collections.deque(range(len(self.tables)))
        gen_event = None
        done = rejected = 0
        nxt = 0
        batch_id = 0
        busy_events = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while done + rejected < N:
            now = time.perf_counter() - t0
            upto = int(np.searchsorted(arrival, now, side="right"))
            if upto > nxt:
                queue.extend(range(nxt, upto))
                nxt = upto
            # admission: FIFO, by device memory
            admitted = []
            while queue:
                i = queue[0]
                if dev_bytes[i] > self.budget:
                    queue.popleft()
                    rejected += 1
                    t_done[i] = np.inf
                    continue
                off = pool.alloc(int(dev_bytes[i]))
                if off is None:
                    break
                queue.popleft()
                offset[i] = off
                admitted.append(i)
            if admitted:
                ids = np.array(admitted)
                t_admit[ids] = time.perf_counter() - t0
                self._generate(addresses(gen_all[ids], ids))
                gen_event = torch.cuda.Event()
                gen_event.record(self.gen_stream)
                ready.extend(admitted)
            # continuous batching: launch whatever is ready when a table is free
            if ready and free_tables:
                k = free_tables.popleft()
                ids = np.array(ready[: self.max_batch])
                ready = ready[self.max_batch:]
                d = addresses(desc_all[ids], ids)
                with torch.cuda.stream(self.exec_stream):
                    self.exec_stream.wait_event(gen_event)
                    start = torch.cuda.Event(enable_timing=True)
                    end = torch.cuda.Event(enable_timing=True)
                    self.tables[k].encode_descs(d.ctypes.data, len(ids))
                    start.record()
                    if self.use_graphs:
                        self._graph_for(k).replay()
                    else:
                        self.tables[k].run()
                    end.record()
                    for i in ids[result_at[ids] >= 0]:
                        c_off = int(offset[i] + a_bytes[i] + s_bytes[i] + x_bytes[i])
                        self.results[result_at[i]:result_at[i] + m[i]].copy_(
                            self.buf[c_off:c_off + 4 * int(m[i])].view(torch.float32))
                    fin = torch.cuda.Event()
                    fin.record()
                t_launch[ids] = time.perf_counter() - t0
                inflight.append((fin, ids, k))
                busy_events.append((start, end))
                batch_id += 1
            # completions
            while inflight and inflight[0][0].query():
                fin, ids, k = inflight.popleft()
                t_done[ids] = time.perf_counter() - t0
                for i in ids:
                    pool.free(int(offset[i]), int(dev_bytes[i]))
                done += len(ids)
                free_tables.append(k)
        torch.cuda.synchronize()
        if warm:
            return None
        for i, r in enumerate(trace):
            r.t_admit, r.t_launch, r.t_done = float(t_admit[i]), float(t_launch[i]), float(t_done[i])
            r.offset, r.result_at = int(offset[i]), int(result_at[i])
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
            batches=nbatches, mean_batch=len(ok) / max(nbatches, 1), total_bytes=total,
            dot_requests=sum(r.op == "dot" for r in ok))

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
