"""Serving loop on the GPU: on-device operand generation equals the host
definition bit for bit; every sampled request of a trace matches the oracle
and is bit-identical when re-run alone; a small HBM budget forces queueing
without changing any result; requests larger than the budget are rejected."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import U32, assert_within, host

pytestmark = pytest.mark.gpu


def host_operands(r):
    """A and x of a request regenerated on the host (SplitMix64 as defined
    in workloads.py; the device kernel implements it separately)."""
    A = workloads.splitmix_uniform(r.seed, 0, r.m * r.n, np.float32).reshape(r.m, r.n)
    x = workloads.splitmix_uniform(r.seed, r.m * r.n, r.n, np.float32)
    return A, x


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("count,seed,c0", [(1, 0, 0), (1000, 7, 5), (1 << 20, 2 ** 63 + 11, 123456789)])
def test_fill_matches_host_generator(sb, dtype, count, seed, c0):
    t = torch.empty(count, dtype=dtype, device="cuda")
    sb.sb_fill_uniform(t, seed, c0)
    ref = workloads.splitmix_uniform(seed, c0, count, np.float32 if dtype == torch.float32 else np.float64)
    assert np.array_equal(host(t), ref)


def check_sampled(sb, server, trace):
    from paper_2108_02025_amd.serve import Request  # noqa: F401
    checked = 0
    for r in trace:
        if r.result_at < 0 or not math.isfinite(r.t_done):
            continue
        got = host(server.result_of(r)).astype(np.float64)
        A, x = host_operands(r)
        if r.op == "dot":
            ref = np.array([oracle.dot(A[0], x, 0.0)])   # alpha = x . y with x = the row, y = the vector
            mag = np.abs(A.astype(np.float64)) @ np.abs(x.astype(np.float64))
        elif r.kind == "f32":
            ref = oracle.gemv(A, x, np.zeros(r.m))
            mag = np.abs(A.astype(np.float64)) @ np.abs(x.astype(np.float64))
        else:
            codes, s = oracle.quantize_rows(A, oracle.Q_BF16)
            ref = oracle.gemv_q(codes, s, x, np.zeros(r.m), oracle.Q_BF16)
            mag = 1.01 * (np.abs(A.astype(np.float64)) @ np.abs(x.astype(np.float64)))
        assert_within(got, ref, 2 * (r.n + 2) * U32 * mag + 1e-30, f"request {r.id} ({r.kind} {r.m}x{r.n})")
        alone = host(server.rerun_alone(r))
        assert np.array_equal(alone, host(server.result_of(r))), f"request {r.id}: alone differs from mix"
        checked += 1
    return checked


def test_serve_trace_matches_oracle_and_alone(sb):
    from paper_2108_02025_amd.serve import Server, make_trace
    trace = make_trace(400, rate=2e4, seed=501, lo=64, hi=2048)
    server = Server(budget_bytes=1 << 30, sample_every=8)
    st = server.run(trace)
    print(st.as_dict())
    assert st.n == 400 and st.rejected == 0 and st.batches >= 1
    assert all(r.t_admit >= r.arrival and r.t_done >= r.t_launch >= r.t_admit for r in trace)
    assert check_sampled(sb, server, trace) == 50


def test_serve_gemv_and_dot_requests(sb):
    """A mixed trace of GEMV and DOT requests (DOTs up to 65536 long, split
    along their length inside the batch): every sampled result matches the
    oracle and is bit-identical alone."""
    from paper_2108_02025_amd.serve import Server, make_trace
    from paper_2108_02025_amd.tuner import TuningTable
    trace = make_trace(240, rate=2e4, seed=909, lo=64, hi=2048, dot_fraction=0.4, dot_hi=65536)
    assert any(r.op == "dot" and r.n > 8192 for r in trace)
    server = Server(budget_bytes=1 << 30, sample_every=3, tuning=TuningTable.load())
    st = server.run(trace)
    print(st.as_dict())
    assert st.n == 240 and st.rejected == 0 and st.dot_requests == sum(r.op == "dot" for r in trace)
    assert check_sampled(sb, server, trace) == 80


def test_serve_full_trace_sampled(sb):
    """The measured serving workload itself (4096 requests, 1e5/s, 4 GiB,
    tuned configurations): every 128th request against the oracle and
    alone."""
    from paper_2108_02025_amd.serve import Server, make_trace
    from paper_2108_02025_amd.tuner import TuningTable
    trace = make_trace(4096, rate=1e5, seed=501)
    server = Server(budget_bytes=4 << 30, sample_every=128, tuning=TuningTable.load())
    st = server.run(trace)
    print(st.as_dict())
    assert st.n == 4096 and st.rejected == 0
    assert check_sampled(sb, server, trace) == 32


def test_serve_small_budget_queues_and_rejects(sb):
    from paper_2108_02025_amd.serve import Request, Server, device_bytes, make_trace
    trace = make_trace(200, rate=5e4, seed=7, lo=64, hi=2048)
    budget = 24 << 20
    big = Request(len(trace), trace[-1].arrival, "f32", 4096, 4096, 99)  # 64 MiB: above the budget
    trace.append(big)
    assert device_bytes("f32", 4096, 4096) > budget
    server = Server(budget_bytes=budget, sample_every=4)
    st = server.run(trace)
    print(st.as_dict())
    assert st.rejected == 1 and not math.isfinite(big.t_done) and st.n == 200
    assert st.batches > 1
    assert check_sampled(sb, server, trace[:200]) == 50


def test_serve_graphs_off_same_bits(sb):
    from paper_2108_02025_amd.serve import Server, make_trace
    outs = []
    for graphs in (True, False):
        trace = make_trace(120, rate=1e4, seed=3, lo=64, hi=1024)
        server = Server(budget_bytes=256 << 20, use_graphs=graphs, sample_every=1)
        server.run(trace)
        outs.append(host(server.results).copy())
    assert np.array_equal(outs[0], outs[1])


def test_servers_share_their_streams(sb):
    """Every Server on a device uses the process's one pair of execution and
    generation streams (two different streams)."""
    from paper_2108_02025_amd.serve import Server
    a, b = Server(budget_bytes=32 << 20, table_bytes=1 << 20), Server(budget_bytes=64 << 20, table_bytes=1 << 20)
    assert a.exec_stream is b.exec_stream and a.gen_stream is b.gen_stream
    assert a.exec_stream.cuda_stream != a.gen_stream.cuda_stream


def test_generate_batched_matches_fill_and_quantise(sb):
    """One sb_generate_batched launch makes the same operands, bit for bit,
    as sb_fill_uniform followed by sb_quantize_rows."""
    import ctypes

    from paper_2108_02025_amd.serve import GEN_DESC, Request, device_bytes, materialise
    # short rows are dealt in blocks of several rows per work item (ragged last blocks)
    shapes = [("f32", 5, 7), ("bf16", 64, 8192), ("bf16", 300, 1000), ("f32", 1000, 300), ("bf16", 3, 0),
              ("f32", 0, 5), ("bf16", 1, 1), ("f32", 700, 64), ("bf16", 513, 33), ("f32", 129, 31),
              ("bf16", 2, 5000), ("f32", 3, 4097),
              # bfloat16 rows past the LDS stash (generated twice), rows on odd counters
              ("bf16", 5, 4097), ("bf16", 3, 8191), ("bf16", 1, 2049), ("bf16", 2, 8193), ("f32", 4, 8193)]
    stage = torch.empty(8192 * 8192, dtype=torch.float32, device="cuda")
    gen = np.zeros(len(shapes), dtype=GEN_DESC)
    bufs, refs = [], []
    for k, (kind, m, n) in enumerate(shapes):
        r = Request(k, 0.0, kind, m, n, 1000 + k)
        b = torch.full((device_bytes(kind, m, n),), 0x5A, dtype=torch.uint8, device="cuda")
        ref = torch.full_like(b, 0x5A)
        materialise(ref, 0, kind, m, n, r.seed, stage)
        es = 4 if kind == "f32" else 2
        up = lambda v: (v + 255) // 256 * 256  # noqa: E731
        a, s_, x = up(es * m * n), up(4 * m) if kind == "bf16" else 0, up(4 * n)
        base = b.data_ptr()
        gen[k] = (2 if kind == "bf16" else 1, 0, m, n, max(n, 1), r.seed, base,
                  base + a if kind == "bf16" else 0, base + a + s_, base + a + s_ + x)
        bufs.append(b)
        refs.append(ref)
    L = sb.load()
    h = sb.Handle()
    h.prepare(int(L.sb_generate_batched_bytes(len(shapes))))
    h.check(L.sb_generate_batched(h.h, ctypes.c_void_p(gen.ctypes.data), len(shapes)))
    torch.cuda.synchronize()
    for (kind, m, n), b, ref in zip(shapes, bufs, refs):
        assert torch.equal(b, ref), (kind, m, n)


def test_generate_batched_padded_rows(sb):
    """With lda > n each row holds the same values as in the packed layout
    and the padding is left untouched."""
    import ctypes

    from paper_2108_02025_amd.serve import GEN_DESC, Request, device_bytes, materialise
    up = lambda v: (v + 255) // 256 * 256  # noqa: E731
    stage = torch.empty(1 << 20, dtype=torch.float32, device="cuda")
    for kind, m, n, pad in (("f32", 37, 100, 3), ("bf16", 37, 100, 5), ("f32", 300, 40, 1), ("bf16", 200, 21, 2),
                            ("bf16", 7, 3001, 3), ("f32", 5, 3001, 1)):
        es = 4 if kind == "f32" else 2
        lda = n + pad
        r = Request(0, 0.0, kind, m, n, 77)
        ref = torch.full((device_bytes(kind, m, n),), 0x5A, dtype=torch.uint8, device="cuda")
        materialise(ref, 0, kind, m, n, r.seed, stage)
        a, s_, x = up(es * m * lda), up(4 * m) if kind == "bf16" else 0, up(4 * n)
        b = torch.full((a + s_ + x + up(4 * m),), 0x5A, dtype=torch.uint8, device="cuda")
        base = b.data_ptr()
        gen = np.zeros(1, dtype=GEN_DESC)
        gen[0] = (2 if kind == "bf16" else 1, 0, m, n, lda, r.seed, base, base + a if s_ else 0, base + a + s_,
                  base + a + s_ + x)
        L = sb.load()
        h = sb.Handle()
        h.prepare(int(L.sb_generate_batched_bytes(1)))
        h.check(L.sb_generate_batched(h.h, ctypes.c_void_p(gen.ctypes.data), 1))
        torch.cuda.synchronize()
        got, want = host(b), host(ref)
        A = got[:es * m * lda].reshape(m, lda * es)
        assert np.array_equal(A[:, :n * es], want[:es * m * n].reshape(m, n * es)), (kind, m, n, lda)
        assert (A[:, n * es:] == 0x5A).all() and (got[es * m * lda:a] == 0x5A).all()
        a0 = up(es * m * n)
        assert np.array_equal(got[a:a + s_ + x + 4 * m], want[a0:a0 + s_ + x + 4 * m]), (kind, m, n, lda)


def test_tuner_quick_and_tuned_serving(sb, tmp_path):
    from paper_2108_02025_amd import tuner
    from paper_2108_02025_amd.serve import Server, make_trace
    data = tuner.tune(buckets={"f32/8/11", "bf16/11/8"}, batch_bytes=8 << 20, log=lambda s: None)
    assert set(data["buckets"]) == {"f32/8/11", "bf16/11/8"}
    for e in data["buckets"].values():
        assert e["us"] <= e["auto_us"] * 1.5 and e["group"] in (4, 8, 16, 32, 64)
    tt = tuner.TuningTable(data)
    assert tt("f32", 256, 2048) == {k: data["buckets"]["f32/8/11"][k] for k in ("group", "rows_per_tile", "split")}
    assert tt("f32", 64, 64) is None
    trace = make_trace(200, rate=2e4, seed=9, lo=128, hi=4096)
    server = Server(budget_bytes=512 << 20, tuning=tt, sample_every=4)
    st = server.run(trace)
    assert st.n == 200
    assert check_sampled(sb, server, trace) == 50


def test_nan_poisoned_request_leaves_every_other_result_unchanged(sb):
    """A request whose x holds a NaN (written after its operands are
    generated, on the generation stream) yields NaN everywhere and leaves
    the bits of every other request of the trace, batched with it,
    unchanged: the batched kernel shares no arithmetic between problems."""
    from paper_2108_02025_amd.serve import GpuExecutor, Server, make_trace

    trace0 = make_trace(160, rate=4e4, seed=31, lo=64, hi=1024)
    victim = next(r.id for r in trace0[40:] if r.kind == "f32" and r.m >= 8)

    class PoisonExecutor(GpuExecutor):
        def generate(self, ids, offset):
            ev = super().generate(ids, offset)
            if victim in ids and not getattr(self, "poisoned", False):
                x_off = int(offset[victim] + self.rel[victim, 2])
                with torch.cuda.stream(self.s.gen_stream):
                    self.s.buf[x_off:x_off + 4].view(torch.float32).fill_(float("nan"))
                ev = torch.cuda.Event()
                ev.record(self.s.gen_stream)
                self.poisoned = True
            return ev

    class PoisonServer(Server):
        executor_class = PoisonExecutor

    def trace_with_burst():
        """The same trace each time, with the victim arriving together with
        its six neighbours so that they share an admission round and a batch."""
        tr = make_trace(160, rate=4e4, seed=31, lo=64, hi=1024)
        for r in tr[victim - 3:victim + 4]:
            r.arrival = tr[victim - 3].arrival
        return tr

    outs = []
    for cls in (Server, PoisonServer):
        trace = trace_with_burst()
        server = cls(budget_bytes=256 << 20, sample_every=1)
        st = server.run(trace, warm_requests=0)
        assert st.n == 160
        outs.append((host(server.results).copy(), trace))
    (clean, t0), (poisoned, t1) = outs
    v = t1[victim]
    sl = slice(v.result_at, v.result_at + v.m)
    assert np.isnan(poisoned[sl]).all() and not np.isnan(clean[sl]).any()
    rest = np.ones(clean.size, bool)
    rest[sl] = False
    assert np.array_equal(clean[rest].view(np.uint32), poisoned[rest].view(np.uint32))
    # the victim shared its batch with other requests
    assert sum(1 for r in t1 if r.t_launch == v.t_launch) > 1
