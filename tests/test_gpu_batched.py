"""Batched persistent GEMV on the GPU: every problem of a random mix against
the oracle, the same problem alone vs in the mix (bitwise), explicit
configurations with split-K, table reuse, and graph replay over new tables."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import U32, U64, assert_within, dev, gamma, gemv_bound, host

pytestmark = pytest.mark.gpu

Q = {"bf16": 2, "e4m3": 3}


def make_problem(sb, rng, kind, m, n, cfg=None, seed=0):
    """Device problem plus the host data the oracle needs."""
    A, x, c0 = workloads.gemv_inputs(m, n, seed=seed, dtype=np.float64 if kind == "f64" else np.float32)
    cfg = cfg or {}
    if kind in ("f64", "f32"):
        P = sb.GemvProblem(dev(A), dev(x), dev(c0), **cfg)
        return P, dict(kind=kind, A=A, x=x, c0=c0)
    q = Q[kind]
    codes, s = oracle.quantize_rows(A, oracle.Q_BF16 if kind == "bf16" else oracle.Q_E4M3)
    cd = dev(codes.view(np.int16) if kind == "bf16" else codes)
    P = sb.GemvProblem(cd, dev(x), dev(c0), scales=dev(s), q=q, **cfg)
    return P, dict(kind=kind, codes=codes, s=s, x=x, c0=c0)


def oracle_check(P, H):
    got = host(P.c).astype(np.float64)
    if H["kind"] in ("f64", "f32"):
        m, n = H["A"].shape
        ref = oracle.gemv(H["A"], H["x"], H["c0"])
        u = U64 if H["kind"] == "f64" else U32
        assert_within(got, ref, gemv_bound(H["A"], H["x"], H["c0"], 0, n, u), H["kind"])
    else:
        qk = oracle.Q_BF16 if H["kind"] == "bf16" else oracle.Q_E4M3
        ref = oracle.gemv_q(H["codes"], H["s"], H["x"], H["c0"], qk)
        dec = np.vectorize(oracle.bf16_to_f32 if qk == oracle.Q_BF16 else oracle.e4m3_to_f32, otypes=[np.float64])
        lut = dec(np.arange(1 << 16 if qk == oracle.Q_BF16 else 256))
        mag = (np.abs(lut[H["codes"]]) * H["s"][:, None].astype(np.float64)) @ np.abs(H["x"].astype(np.float64))
        n = H["codes"].shape[1]
        bound = 2 * (n + 2) * U32 * (np.abs(H["c0"]) + mag) + 1e-30
        assert_within(got, ref, bound, H["kind"])


def fresh_copy(sb, P, H):
    """The same problem with its own output vector reset to c0."""
    return sb.GemvProblem(P.A, P.x, dev(H["c0"]), scales=P.scales, q=P.q, group=P.group,
                          rows_per_tile=P.rows_per_tile, split=P.split, op=P.op)


def test_batched_random_mix_alone_vs_mix(sb):
    rng = np.random.default_rng(501)
    kinds = ["f64", "f32", "bf16", "e4m3"]
    probs, hosts = [], []
    for i in range(40):
        m = int(np.exp(rng.uniform(np.log(1), np.log(3000))))
        n = int(np.exp(rng.uniform(np.log(1), np.log(9000))))
        P, H = make_problem(sb, rng, kinds[i % 4], m, n, seed=1000 + i)
        probs.append(P)
        hosts.append(H)
    sb.sb_gemv_batched(probs)
    mix = [host(P.c).copy() for P in probs]
    for P, H, got in zip(probs, hosts, mix):
        oracle_check(P, H)
        alone = fresh_copy(sb, P, H)
        sb.sb_gemv_batched([alone])
        assert np.array_equal(host(alone.c), got), "alone differs from mix"


@pytest.mark.parametrize("cfg", [dict(group=4, rows_per_tile=64, split=1), dict(group=16, rows_per_tile=16, split=3),
                                 dict(group=64, rows_per_tile=8, split=2), dict(group=32, rows_per_tile=0, split=5),
                                 dict(group=8, rows_per_tile=32, split=0)])
@pytest.mark.parametrize("kind", ["f64", "f32", "bf16", "e4m3"])
def test_batched_configs(sb, cfg, kind):
    rng = np.random.default_rng(7)
    probs, hosts = [], []
    for i, (m, n) in enumerate([(1, 5), (37, 1000), (300, 4099), (1025, 33), (64, 8192), (5, 20000)]):
        max_kc = 4096 if kind == "f64" else 8192  # x chunk of a tile: 32 KiB of LDS
        sp = cfg.get("split") or 0
        if sp and -(-(-(-n // sp)) // 16) * 16 > max_kc:
            continue  # this split leaves a chunk too wide for LDS (rejected by design)
        P, H = make_problem(sb, rng, kind, m, n, cfg=cfg, seed=i)
        probs.append(P)
        hosts.append(H)
    sb.sb_gemv_batched(probs)
    for P, H in zip(probs, hosts):
        oracle_check(P, H)
    # the same problems again in reverse order with fresh outputs: same bits
    again = [fresh_copy(sb, P, H) for P, H in zip(probs, hosts)][::-1]
    sb.sb_gemv_batched(again)
    for P, Q2 in zip(probs, again[::-1]):
        assert torch.equal(P.c, Q2.c)


def test_batched_integer_exact_and_table_reuse(sb):
    """Integer data is exact; launching the same table twice adds A x twice
    (split counters re-arm themselves)."""
    rng = np.random.default_rng(3)
    probs, refs = [], []
    for i, (m, n) in enumerate([(100, 3000), (7, 9000), (513, 513)]):
        A, x, c0 = workloads.gemv_inputs(m, n, seed=i, dist="int8")
        P = sb.GemvProblem(dev(A), dev(x), dev(c0), split=3)
        probs.append(P)
        refs.append((A.astype(np.int64), x.astype(np.int64), c0))
    table = sb.BatchTable(sb.sb_gemv_batched_table_bytes(probs)[0])
    table.encode(probs)
    table.run()
    table.run()
    for P, (A, x, c0) in zip(probs, refs):
        assert np.array_equal(host(P.c), c0 + 2 * (A @ x))


def test_batched_graph_replay(sb):
    """A captured launch replayed over new tables written to the same
    address gives the eager results, replay after replay."""
    rng = np.random.default_rng(11)
    batches = []
    for b in range(3):
        ps, hs = [], []
        for i in range(6):
            m, n = int(rng.integers(1, 900)), int(rng.integers(1, 5000))
            P, H = make_problem(sb, rng, ["f32", "bf16"][i % 2], m, n, seed=100 * b + i)
            ps.append(P)
            hs.append(H)
        batches.append((ps, hs))
    cap = max(sb.sb_gemv_batched_table_bytes(ps)[0] for ps, _ in batches)
    table = sb.BatchTable(cap)
    eager = []
    for ps, hs in batches:
        fresh = [fresh_copy(sb, P, H) for P, H in zip(ps, hs)]
        sb.sb_gemv_batched(fresh)
        eager.append([host(P.c).copy() for P in fresh])
    table.encode(batches[0][0])
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        table.run()                       # warm-up outside capture
        torch.cuda.synchronize()
        for P, H in zip(*batches[0]):
            P.c.copy_(dev(H["c0"]))
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            table.run()
    torch.cuda.synchronize()
    for rep in range(2):
        for (ps, hs), ref in zip(batches, eager):
            for P, H in zip(ps, hs):
                P.c.copy_(dev(H["c0"]))
            table.encode(ps)
            graph.replay()
            torch.cuda.synchronize()
            for P, r in zip(ps, ref):
                assert np.array_equal(host(P.c), r), f"replay {rep}"


def test_batched_rejects_bad_input(sb):
    A = torch.zeros((10, 10), dtype=torch.float32, device="cuda")
    x = torch.zeros(10, dtype=torch.float32, device="cuda")
    c = torch.zeros(10, dtype=torch.float32, device="cuda")
    with pytest.raises(sb.StreamBlasError):
        sb.sb_gemv_batched_resolve([sb.GemvProblem(A, x, c, group=3)])
    with pytest.raises(sb.StreamBlasError):
        sb.sb_gemv_batched_resolve([sb.GemvProblem(A, x, c), sb.GemvProblem(A, x, c)])  # shared output
    with pytest.raises(sb.StreamBlasError):
        sb.sb_gemv_batched_resolve([sb.GemvProblem(A, x, c, group=64, rows_per_tile=3)])
    r = sb.sb_gemv_batched_resolve([sb.GemvProblem(A, x, c)])
    assert r[0]["split"] == 1 and r[0]["group"] in (4, 8, 16, 32, 64)


def test_plan_runs_match_batched_and_replay(sb):
    """A plan gives the one-call batched results bit for bit, run after run
    (each run adds A x again), also from a captured graph replayed with
    eager work in between."""
    rng = np.random.default_rng(77)
    probs, hosts = [], []
    for i in range(12):
        m, n = int(rng.integers(1, 2000)), int(rng.integers(1, 12000))
        P, H = make_problem(sb, rng, ["f64", "f32", "bf16", "e4m3"][i % 4], m, n, seed=300 + i)
        probs.append(P)
        hosts.append(H)
    ref = [fresh_copy(sb, P, H) for P, H in zip(probs, hosts)]
    for _ in range(3):
        sb.sb_gemv_batched(ref)
    want = [host(P.c).copy() for P in ref]
    plan = sb.Plan(probs)
    for _ in range(3):
        plan.run()
    assert all(np.array_equal(host(P.c), w) for P, w in zip(probs, want))
    # graph replays: reset c, replay three times with eager GEMVs between
    for P, H in zip(probs, hosts):
        P.c.copy_(dev(H["c0"]))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.run()
    torch.cuda.synchronize()
    for P, H in zip(probs, hosts):
        P.c.copy_(dev(H["c0"]))
    other = torch.ones((300, 300), dtype=torch.float64, device="cuda")
    for _ in range(3):
        g.replay()
        sb.sb_gemv(other, torch.ones(300, dtype=torch.float64, device="cuda"),
                   torch.zeros(300, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
    assert all(np.array_equal(host(P.c), w) for P, w in zip(probs, want))


def test_plan_invalidated_by_workspace_writes(sb):
    """Through the C-ABI: a call that writes the handle's workspace (a
    two-stage DOT) makes sb_plan_run fail until the plan is made again; a
    call that needs no workspace leaves it valid."""
    import ctypes
    L = sb.load()
    rng = np.random.default_rng(5)
    P, H = make_problem(sb, rng, "f32", 300, 700, seed=9)
    descs = sb.make_descs([P])
    total, _ = sb.sb_gemv_batched_table_bytes([P])
    ws = torch.empty(max(total, 1 << 22), dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.sb_handle_create(ctypes.c_void_p(ws.data_ptr()), ws.numel(), stream, ctypes.byref(h)) == 0
    p = ctypes.c_void_p()
    try:
        assert L.sb_plan_create(h, descs, 1, ctypes.byref(p)) == 0
        assert L.sb_plan_run(p) == 0
        x = torch.rand(1 << 20, dtype=torch.float64, device="cuda")
        a = torch.zeros(1, dtype=torch.float64, device="cuda")
        assert L.sb_dot(h, 0, 100, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                        ctypes.c_void_p(a.data_ptr())) == 0           # small: no workspace
        assert L.sb_plan_run(p) == 0
        assert L.sb_dot(h, 0, 1 << 20, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                        ctypes.c_void_p(a.data_ptr())) == 0           # two-stage: writes the workspace
        assert L.sb_plan_run(p) == -1 and b"create the plan again" in L.sb_last_error(h)
        assert L.sb_plan_destroy(p) == 0
        assert L.sb_plan_create(h, descs, 1, ctypes.byref(p)) == 0 and L.sb_plan_run(p) == 0
        torch.cuda.synchronize()
        got = host(P.c).astype(np.float64)
        ref = oracle.gemv(H["A"], H["x"], H["c0"])
        ref = oracle.gemv(H["A"], H["x"], oracle.gemv(H["A"], H["x"], ref))   # three runs in all
        assert_within(got, ref, 6 * gemv_bound(H["A"], H["x"], np.abs(H["c0"]) + 3 * np.abs(ref), 0, 700, U32), "plan")
    finally:
        L.sb_plan_destroy(p)
        L.sb_handle_destroy(h)


# ----------------------------------------------------- layouts and ops ----
# (row-major, N) and (column-major, T) are row dots over the stored rows;
# (row-major, T) and (column-major, N) are column axpys over them.

LAYOUT_OPS = [(0, 0), (1, 1), (0, 1), (1, 0)]


def stored(A, layout, pad=0):
    """Device tensor of logical shape A.shape stored row- or column-major,
    each stored row followed by `pad` NaN elements (so a read outside the
    matrix would poison the result, and pad > 0 moves the rows off 16-byte
    alignment)."""
    S = A if layout == 0 else A.T
    buf = np.full((S.shape[0], S.shape[1] + pad), np.nan, dtype=A.dtype)
    buf[:, :S.shape[1]] = S
    d = dev(buf)[:, :S.shape[1]]
    return d if layout == 0 else d.t()


def test_batched_layouts_and_ops_mix(sb):
    """Every (layout, op) pair in binary64 and binary32, with aligned and
    unaligned stored rows and edge shapes, in one batch: each problem within
    the summation bound of the oracle, and alone gives the bits it gave in
    the mix."""
    shapes = [(1, 1), (1, 300), (300, 1), (37, 1000), (1000, 37), (257, 513), (2048, 3000), (5, 20000),
              (20000, 5)]
    probs, hosts = [], []
    k = 0
    for kind, npd, u in (("f64", np.float64, U64), ("f32", np.float32, U32)):
        for m, n in shapes:
            for layout, op in LAYOUT_OPS:
                A, x, c0 = workloads.gemv_inputs(m, n, seed=2000 + k, dist="normal", op_t=bool(op), dtype=npd)
                P = sb.GemvProblem(stored(A, layout, pad=k % 3), dev(x), dev(c0), op=op)
                probs.append(P)
                hosts.append(dict(A=A, x=x, c0=c0, op=op, u=u, what=f"{kind} {m}x{n} layout {layout} op {op}"))
                k += 1
    sb.sb_gemv_batched(probs)
    mix = [host(P.c).copy() for P in probs]
    for P, H, got in zip(probs, hosts, mix):
        m, n = H["A"].shape
        ref = oracle.gemv(H["A"], H["x"], H["c0"], op=H["op"])
        K = n if H["op"] == 0 else m
        assert_within(got, ref, gemv_bound(H["A"], H["x"], H["c0"], H["op"], K, H["u"]), H["what"])
        alone = fresh_copy(sb, P, H)
        sb.sb_gemv_batched([alone])
        assert np.array_equal(host(alone.c), got), "alone differs from mix: " + H["what"]


@pytest.mark.parametrize("cfg", [dict(rows_per_tile=1), dict(rows_per_tile=7), dict(split=3), dict(split=1),
                                 dict(rows_per_tile=200, split=5)])
@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_batched_column_axpy_chunks_exact_and_table_reuse(sb, kind, cfg):
    """Column axpys with explicit row chunking on integer data (every sum
    exact): the oracle's bits, and a table launched twice adds op(A) x
    twice (the chunk counters re-arm themselves)."""
    npd = np.float64 if kind == "f64" else np.float32
    probs, refs = [], []
    for i, (m, n, layout, pad) in enumerate([(1000, 300, 0, 0), (999, 1001, 0, 1), (300, 1000, 1, 0),
                                             (1001, 999, 1, 3), (1, 70, 0, 0)]):
        op = 1 if layout == 0 else 0      # the column-axpy pairs
        rows = m if layout == 0 else n    # stored rows
        if cfg.get("rows_per_tile") and cfg.get("split") and -(-rows // cfg["rows_per_tile"]) != cfg["split"]:
            continue                      # chunking that disagrees is rejected (CPU test)
        A, x, c0 = workloads.gemv_inputs(m, n, seed=40 + i, dist="int8" if kind == "f64" else "int7",
                                         op_t=bool(op), dtype=npd)
        P = sb.GemvProblem(stored(A, layout, pad), dev(x), dev(c0), op=op, **cfg)
        probs.append(P)
        r = oracle.gemv(A, x, c0, op=op)
        refs.append((r, c0 + 2 * (r - c0)))
    for P, r in zip(probs, sb.sb_gemv_batched_resolve(probs)):
        assert r["group"] == 0
        if cfg.get("rows_per_tile"):
            assert r["rows_per_tile"] == cfg["rows_per_tile"]
    table = sb.BatchTable(sb.sb_gemv_batched_table_bytes(probs)[0])
    table.encode(probs)
    table.run()
    torch.cuda.synchronize()
    for P, (once, _) in zip(probs, refs):
        assert np.array_equal(host(P.c), once)
    table.run()
    for P, (_, twice) in zip(probs, refs):
        assert np.array_equal(host(P.c), twice)


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_batched_same_buffer_pairs_bitwise(sb, kind):
    """On one buffer, (row-major, T) and (column-major, N) are the same
    computation and give the same bits; so are (row-major, N) and
    (column-major, T); the batch matches the single-call sb_gemv to the
    summation bound."""
    npd, u = (np.float64, U64) if kind == "f64" else (np.float32, U32)
    m, n = 777, 1531
    A, _, _ = workloads.gemv_inputs(m, n, seed=5, dist="normal", dtype=npd)
    buf = dev(A)
    colview = buf.reshape(-1).as_strided((n, m), (1, n))     # the same memory as an n x m column-major matrix
    xm = dev(workloads.gemv_inputs(m, 1, seed=6, dtype=npd)[0].reshape(-1))
    xn = dev(workloads.gemv_inputs(n, 1, seed=7, dtype=npd)[0].reshape(-1))
    cm = [dev(np.zeros(m, npd)) for _ in range(2)]
    cn = [dev(np.zeros(n, npd)) for _ in range(2)]
    sb.sb_gemv_batched([sb.GemvProblem(buf, xm, cn[0], op=1), sb.GemvProblem(colview, xm, cn[1], op=0),
                        sb.GemvProblem(buf, xn, cm[0], op=0), sb.GemvProblem(colview, xn, cm[1], op=1)])
    assert torch.equal(cn[0], cn[1]) and torch.equal(cm[0], cm[1])
    Ah = A.astype(np.float64)
    for got, ref, bnd in ((cn[0], Ah.T @ host(xm), 2 * gamma(m + 1, u) * (np.abs(Ah).T @ np.abs(host(xm)))),
                          (cm[0], Ah @ host(xn), 2 * gamma(n + 1, u) * (np.abs(Ah) @ np.abs(host(xn))))):
        assert np.all(np.abs(host(got) - ref) <= bnd + 1e-300)


def test_batched_quantised_layouts_rejected(sb):
    codes = torch.zeros((10, 10), dtype=torch.int16, device="cuda")
    s = torch.ones(10, dtype=torch.float32, device="cuda")
    x = torch.zeros(10, dtype=torch.float32, device="cuda")
    c = torch.zeros(10, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        sb.make_descs([sb.GemvProblem(codes, x, c, scales=s, q=sb.SB_BF16, op=sb.SB_T)])
    with pytest.raises(ValueError):
        sb.make_descs([sb.GemvProblem(codes.t(), x, c, scales=s, q=sb.SB_BF16)])


def test_batched_graph_replay_split_and_column_problems(sb):
    """A captured run replayed over new tables whose problems need the second
    stage (split row dots, chunked column axpys) or none: every replay gives
    the eager bits, with eager work on the same stream between replays."""
    rng = np.random.default_rng(21)
    batches = []
    for b in range(3):
        ps, hs = [], []
        for i in range(5):
            kind = ["f64", "f32"][i % 2]
            npd = np.float64 if kind == "f64" else np.float32
            m, n = int(rng.integers(1, 700)), int(rng.integers(1, 9000))
            layout, op = LAYOUT_OPS[(b + i) % 4]
            A, x, c0 = workloads.gemv_inputs(m, n, seed=700 + 10 * b + i, dist="normal", op_t=bool(op), dtype=npd)
            cfg = {} if b == 2 else ({"split": 3} if (layout, op) in ((0, 0), (1, 1)) else {"rows_per_tile": 37})
            ps.append(sb.GemvProblem(stored(A, layout, pad=i % 2), dev(x), dev(c0), op=op, **cfg))
            hs.append(dict(c0=c0))
        batches.append((ps, hs))
    cap = max(sb.sb_gemv_batched_table_bytes(ps)[0] for ps, _ in batches)
    table = sb.BatchTable(cap)
    eager = []
    for ps, hs in batches:
        fresh = [sb.GemvProblem(P.A, P.x, dev(H["c0"]), op=P.op, group=P.group, rows_per_tile=P.rows_per_tile,
                                split=P.split) for P, H in zip(ps, hs)]
        sb.sb_gemv_batched(fresh)
        eager.append([host(P.c).copy() for P in fresh])
    table.encode(batches[0][0])
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        table.run()
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            table.run()
    torch.cuda.synchronize()
    other = torch.ones((300, 300), dtype=torch.float64, device="cuda")
    for rep in range(2):
        for (ps, hs), ref in zip(batches, eager):
            for P, H in zip(ps, hs):
                P.c.copy_(dev(H["c0"]))
            table.encode(ps)
            graph.replay()
            sb.sb_gemv(other, torch.ones(300, dtype=torch.float64, device="cuda"),
                       torch.zeros(300, dtype=torch.float64, device="cuda"))
            torch.cuda.synchronize()
            for P, r in zip(ps, ref):
                assert np.array_equal(host(P.c), r), f"replay {rep}"
