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
    A = workloads.splitmix_uniform(r.seed, 0, r.m * r.n).astype(np.float32).reshape(r.m, r.n)
    x = workloads.splitmix_uniform(r.seed, r.m * r.n, r.n).astype(np.float32)
    return A, x


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("count,seed,c0", [(1, 0, 0), (1000, 7, 5), (1 << 20, 2 ** 63 + 11, 123456789)])
def test_fill_matches_host_generator(sb, dtype, count, seed, c0):
    t = torch.empty(count, dtype=dtype, device="cuda")
    sb.sb_fill_uniform(t, seed, c0)
    ref = workloads.splitmix_uniform(seed, c0, count)
    ref = ref.astype(np.float32) if dtype == torch.float32 else ref
    assert np.array_equal(host(t), ref)


def check_sampled(sb, server, trace):
    from paper_2108_02025_amd.serve import Request  # noqa: F401
    checked = 0
    for r in trace:
        if r.result_at < 0 or not math.isfinite(r.t_done):
            continue
        got = host(server.result_of(r)).astype(np.float64)
        A, x = host_operands(r)
        if r.kind == "f32":
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
