#!/usr/bin/env python3
"""Throughput of the streaming GEMV / DOT / GER hot path on one MI355X.

One step is one pass over every operation of the hot path, each on its full
size, operands resident in HBM before timing starts:

  gemv_n_f64   c += A x,    A 16384 x 16384 binary64 row-major, uniform[-1,1)
  gemv_t_f64   c += A^T x,  same A
  gemv2_f64    c += A x and d += A^T y in one pass over the same A
  dot_f64      alpha += x . y, n = 2^28 binary64
  ger_f64      C += x (outer) y, C 16384 x 16384 binary64
  gemv_q_bf16  c += diag(s) Q x, Q = bfloat16 codes of A (per-row scales), x binary32
  gemv_q_e4m3  the same with OCP E4M3FN codes
  gemv_mx_fp8  c += A x with A as MXFP8 (E4M3 codes, one E8M0 scale per 32)
  gemv_mx_fp4  the same with MXFP4 (E2M1 codes)
  dot2_f32     compensated binary32 dot, n = 2^27, condition number 1e8

(quantisation of A is a one-off pre-step and is not timed).  ``value`` is the
aggregate algorithmic HBM throughput of the step: the bytes each operation
must move (every operand element touched once) summed over the step, divided
by the step time.  Per-operation times come from HIP events recorded on the
stream the library launches on, one between consecutive operations, created
without the system-scope fence (``--fenced-events`` uses default events).

Besides the step, the JSON line reports the HBM read/copy ceilings, small
problem latencies (``small``), the GEMVs on the skewed shapes 262144x256,
256x262144, 65536x4096 and 65537x4093 in binary64 and binary32
(``skewed``), the serving trace (``serving``) and the CPU oracle baseline.

    python bench.py [--steps K] [--warmup W] [--no-cpu] [--no-serve] [--no-small] [--no-skewed] [--ops a,b]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC = os.path.join(HERE, "profiles", "hbm_traffic.json")

# Source files whose contents determine each operation's kernels; measured
# traffic is reported only while their hash matches the one recorded with it.
KERNEL_SOURCES = {
    "gemv_n_f64": ["gemv.hip", "sb_rowdot.hpp", "sb_device.hpp"],
    "gemv_t_f64": ["gemv.hip", "sb_device.hpp"],
    "gemv2_f64": ["gemv2.hip", "sb_wave.hpp", "sb_device.hpp"],
    "dot_f64": ["dot.hip", "sb_device.hpp"],
    "ger_f64": ["ger.hip", "sb_device.hpp"],
    "gemv_q_bf16": ["quant.hip", "sb_rowdot.hpp", "sb_quant.hpp", "sb_device.hpp"],
    "gemv_q_e4m3": ["quant.hip", "sb_rowdot.hpp", "sb_quant.hpp", "sb_device.hpp"],
    "dot2_f32": ["dot.hip", "sb_device.hpp"],
    "gemv_mx_fp8": ["mx.hip", "sb_quant.hpp", "sb_device.hpp"],
    "gemv_mx_fp4": ["mx.hip", "sb_quant.hpp", "sb_device.hpp"],
}


def source_hash(op: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[op]:
        with open(os.path.join(HERE, "paper_2108_02025_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(op: str):
    """HBM bytes per call from the committed counter measurement, or None
    when there is none or the kernel sources changed since it was taken."""
    if not os.path.exists(TRAFFIC) or op not in KERNEL_SOURCES:
        return None
    with open(TRAFFIC) as f:
        d = json.load(f)
    e = d.get("ops", {}).get(op)
    if not e or e.get("source_sha256") != source_hash(op):
        return None
    return e["traffic_bytes"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_ops(sb, torch, dev, sel):
    """Operands on the device and the list of (name, bytes, flops, fn)."""
    import workloads  # noqa: F401  (host recipes; device draws below follow the same distributions)

    M = N = 16384
    nd = 1 << 28
    n2 = 1 << 27
    g = torch.Generator(device=dev)

    def uni(shape, seed, dtype=torch.float64):
        g.manual_seed(seed)
        return (torch.rand(shape, generator=g, device=dev, dtype=dtype) * 2 - 1)

    ops = []
    want = (lambda name: sel is None or name in sel)
    A = None
    if any(want(k) for k in ("gemv_n_f64", "gemv_t_f64", "gemv2_f64", "gemv_q_bf16", "gemv_q_e4m3", "gemv_mx_fp8",
                             "gemv_mx_fp4")):
        log("drawing A 16384x16384 binary64")
        A = uni((M, N), 201)
    if want("gemv_n_f64"):
        x, c = uni((N,), 2011), uni((M,), 2012)
        ops.append(("gemv_n_f64", 8 * (M * N + N + 2 * M), 2 * M * N, lambda: sb.sb_gemv(A, x, c, op=sb.SB_N),
                    {"kind": "gemv", "A": A, "x": x, "c": c, "op": 0}))
    if want("gemv_t_f64"):
        xt, ct = uni((M,), 2013), uni((N,), 2014)
        ops.append(("gemv_t_f64", 8 * (M * N + M + 2 * N), 2 * M * N, lambda: sb.sb_gemv(A, xt, ct, op=sb.SB_T),
                    {"kind": "gemv", "A": A, "x": xt, "c": ct, "op": 1}))
    if want("gemv2_f64"):
        x2, y2, c2, d2 = uni((N,), 2015), uni((M,), 2016), uni((M,), 2017), uni((N,), 2018)
        ops.append(("gemv2_f64", 8 * (M * N + N + M + 2 * M + 2 * N), 4 * M * N,
                    lambda: sb.sb_gemv2(A, x2, y2, c2, d2), {"kind": "gemv2", "A": A, "x": x2, "y": y2, "c": c2, "d": d2}))
    if want("dot_f64"):
        log("drawing DOT vectors n=2^28")
        dx, dy, da = uni((nd,), 2021), uni((nd,), 2022), uni((1,), 2023)
        ops.append(("dot_f64", 8 * (2 * nd + 2), 2 * nd, lambda: sb.sb_dot(dx, dy, da),
                    {"kind": "dot", "x": dx, "y": dy, "a": da}))
    if want("ger_f64"):
        log("drawing GER operands 16384x16384")
        gx, gy, gC = uni((M,), 2031), uni((N,), 2032), uni((M, N), 2033)
        ops.append(("ger_f64", 8 * (2 * M * N + M + N), 2 * M * N, lambda: sb.sb_ger(gx, gy, gC),
                    {"kind": "ger", "x": gx, "y": gy, "C": gC}))
    for q, name, es in ((sb.SB_BF16, "gemv_q_bf16", 2), (sb.SB_FP8_E4M3, "gemv_q_e4m3", 1)):
        if not want(name):
            continue
        log(f"quantising A for {name} (untimed pre-step)")
        A32 = A.float()
        Aq = torch.empty((M, N), dtype=torch.int16 if es == 2 else torch.uint8, device=dev)
        s = torch.empty(M, dtype=torch.float32, device=dev)
        sb.sb_quantize_rows(A32, Aq, s, q)
        del A32
        g.manual_seed(401)
        xq = torch.randn(N, generator=g, device=dev, dtype=torch.float32)
        cq = torch.zeros(M, dtype=torch.float32, device=dev)
        ops.append((name, es * M * N + 4 * N + 8 * M + 4 * M, 2 * M * N,
                    (lambda Aq=Aq, s=s, xq=xq, cq=cq, q=q: sb.sb_gemv_q(Aq, s, xq, cq, q)),
                    {"kind": "gemv_q", "A": A, "Q": Aq, "s": s, "x": xq, "c": cq, "q": q}))
    for q, name, rb in ((sb.SB_MXFP8_E4M3, "gemv_mx_fp8", N), (sb.SB_MXFP4_E2M1, "gemv_mx_fp4", N // 2)):
        if not want(name):
            continue
        log(f"MX-quantising A for {name} (untimed pre-step)")
        A32 = A.float()
        Q, S = sb.mx_buffers(q, M, N, dev)
        sb.sb_quantize_mx(A32, Q, S, q)
        del A32
        g.manual_seed(402)
        xm = torch.randn(N, generator=g, device=dev, dtype=torch.float32)
        cm = torch.zeros(M, dtype=torch.float32, device=dev)
        ops.append((name, M * rb + M * (N // 32) + 4 * N + 8 * M, 2 * M * N,
                    (lambda Q=Q, S=S, xm=xm, cm=cm, q=q: sb.sb_gemv_mx(Q, S, xm, cm, q)),
                    {"kind": "gemv_mx", "A": A, "Q": Q, "S": S, "x": xm, "c": cm, "q": q}))
    if want("dot2_f32"):
        log("generating ill-conditioned pairs n=2^27 (cond 1e8)")
        import workloads
        hx, hy, ha, cond = workloads.illcond_dot_inputs(n2, seed=402)
        ex, ey = torch.from_numpy(hx).to(dev), torch.from_numpy(hy).to(dev)
        ea = torch.zeros(1, dtype=torch.float32, device=dev)
        ops.append(("dot2_f32", 4 * (2 * n2 + 2), 2 * n2, lambda: sb.sb_dot2_f32(ex, ey, ea),
                    {"kind": "dot2", "x": ex, "y": ey, "hx": hx, "hy": hy, "cond": cond}))
    torch.cuda.synchronize()
    return ops


def build_probes(sb, torch, dev):
    """Streaming read of 4 GiB and copy of 2 GiB with the library's probes:
    the practical HBM ceilings the operations are compared against."""
    src = torch.empty(1 << 29, dtype=torch.float64, device=dev)   # 4 GiB
    src.fill_(1.0)
    half = src[: 1 << 28]
    dst = torch.empty(1 << 28, dtype=torch.float64, device=dev)   # 2 GiB
    upd = src[: 1 << 28].view(16384, 16384)                       # GER's matrix shape, 2 GiB
    return [("probe_read", 8 << 29, 0, lambda: sb.sb_stream_read(src)),
            ("probe_copy", 2 * (8 << 28), 0, lambda: sb.sb_stream_copy(half, dst)),
            ("probe_update", 2 * (8 << 28), 0, lambda: sb.sb_stream_update(upd))]


class HipEvents:
    """HIP timing events recorded on the stream the library launches on
    (torch's current stream).  By default they are created with
    hipEventDisableSystemFence: such an event only takes a GPU timestamp,
    without the system-scope release (cache write-back and invalidation)
    that a default event performs when it completes, whose cost would
    otherwise fall into the window of the operation that follows it.
    Kernels on the stream still run strictly one after another."""

    DISABLE_SYSTEM_FENCE = 0x20000000

    def __init__(self, torch, fence=False):
        import ctypes

        from paper_2108_02025_amd.build import torch_lib_dir
        self.ct = ctypes
        self.hip = ctypes.CDLL(os.path.join(torch_lib_dir(), "libamdhip64.so"))
        self.hip.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        self.hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.flags = 0 if fence else self.DISABLE_SYSTEM_FENCE
        self.torch = torch
        self.events = []

    def _check(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"{what} failed with HIP error {rc}")

    def record(self):
        ev = self.ct.c_void_p()
        self._check(self.hip.hipEventCreateWithFlags(self.ct.byref(ev), self.flags), "hipEventCreateWithFlags")
        self.events.append(ev)
        stream = self.torch.cuda.current_stream().cuda_stream
        self._check(self.hip.hipEventRecord(ev, self.ct.c_void_p(stream)), "hipEventRecord")
        return ev

    def ms(self, a, b):
        out = self.ct.c_float()
        self._check(self.hip.hipEventElapsedTime(self.ct.byref(out), a, b), "hipEventElapsedTime")
        return out.value

    def close(self):
        for ev in self.events:
            self.hip.hipEventDestroy(ev)
        self.events = []


def time_ops(torch, ops, steps, fence=False):
    """Per-operation times (us) over `steps` passes, and the step time (ms).
    One event is recorded between consecutive operations, so an operation's
    window runs from the event before it to the event after it."""
    ev = HipEvents(torch, fence)
    per = {n: [] for n, *_ in ops}
    torch.cuda.synchronize()
    marks = [ev.record()]
    for _ in range(steps):
        for name, _, _, fn, *_ in ops:
            fn()
            marks.append(ev.record())
    torch.cuda.synchronize()
    k = 0
    for _ in range(steps):
        for name, *_ in ops:
            per[name].append(ev.ms(marks[k], marks[k + 1]))
            k += 1
    total = ev.ms(marks[0], marks[-1])
    ev.close()
    return {n: 1e3 * sum(v) / len(v) for n, v in per.items()}, total / steps


def cpu_baseline(step_bytes, thread_counts=(1,)):
    """The CPU oracle, as it stands, on the step's operations: binary64 GEMV
    N/T, the two-sided GEMV and GER on the full 16384 x 16384 size and DOT
    on the full 2^28; the quantised GEMVs on 4096 rows, the MX GEMVs on 1024
    and the exact dot on 2^24 pairs.  With threads > 1 each call is cut into that many
    disjoint row slices (chunks for the dots) run concurrently (the oracle's
    C code releases the interpreter lock); slices of a column sum are added
    afterwards, which is enough for timing.  Each operation's rate is applied
    to the full step's bytes.  Returns one result per thread count; the
    inputs are drawn once."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    import workloads

    oracle.build()
    M = N = 16384
    rates = {t: {} for t in thread_counts}
    parts = {t: [] for t in thread_counts}
    pools = {t: ThreadPoolExecutor(t) for t in thread_counts}

    def timed(name, nbytes, fn, n):
        """fn(a, b) runs the oracle on rows (or elements) [a, b)."""
        for t in thread_counts:
            b = np.linspace(0, n, t + 1).astype(int)
            t0 = time.perf_counter()
            list(pools[t].map(lambda ab: fn(*ab), zip(b[:-1], b[1:])))
            dt = time.perf_counter() - t0
            rates[t][name] = nbytes / dt
            parts[t].append(f"{name}:{nbytes / 1e6:.0f}MB/{dt:.2f}s")
            log(f"oracle x{t} {name}: {nbytes / dt / 1e9:.2f} GB/s")

    A, x, c0 = workloads.gemv_inputs(M, N, seed=201)
    y2, d0 = np.ones(M), np.zeros(N)
    timed("gemv_n_f64", 8 * (M * N + N + 2 * M), lambda a, b: oracle.gemv(A[a:b], x, c0[a:b]), M)
    timed("gemv_t_f64", 8 * (M * N + M + 2 * N),
          lambda a, b: oracle.gemv(A[a:b], x[a:b], c0, op=oracle.OP_T), M)
    timed("gemv2_f64", 8 * (M * N + 3 * M + 3 * N),
          lambda a, b: oracle.gemv2(A[a:b], x, y2[a:b], c0[a:b], d0), M)
    rows = 4096
    A32 = np.ascontiguousarray(A[:rows]).astype(np.float32)
    del A
    xq = np.random.default_rng(401).standard_normal(N).astype(np.float32)
    for q, name, es in ((oracle.Q_BF16, "gemv_q_bf16", 2), (oracle.Q_E4M3, "gemv_q_e4m3", 1)):
        codes, s = oracle.quantize_rows(A32, q)
        timed(name, es * rows * N + 4 * N + 12 * rows,
              lambda a, b: oracle.gemv_q(codes[a:b], s[a:b], xq, np.zeros(b - a), q), rows)
    mrows = 1024
    for q, name, rb in ((oracle.Q_MXFP8, "gemv_mx_fp8", N), (oracle.Q_MXFP4, "gemv_mx_fp4", N // 2)):
        codes, s = oracle.quantize_mx(A32[:mrows], q)
        timed(name, mrows * rb + mrows * (N // 32) + 4 * N + 8 * mrows,
              lambda a, b: oracle.gemv_mx(codes[a:b], s[a:b], xq, np.zeros(b - a), q, N), mrows)
    del A32
    nd = 1 << 28
    dx, dy, da = workloads.dot_inputs(nd, seed=202)
    timed("dot_f64", 8 * (2 * nd + 2), lambda a, b: oracle.dot(dx[a:b], dy[a:b], da[0]), nd)
    del dx, dy
    gx, gy, gC = workloads.ger_inputs(M, N, seed=203)
    timed("ger_f64", 8 * (2 * M * N + M + N), lambda a, b: oracle.ger(gx[a:b], gy, gC[a:b]), M)
    del gC
    n2 = 1 << 24
    hx, hy, _, _ = workloads.illcond_dot_inputs(n2, seed=402)
    timed("dot2_f32", 4 * (2 * n2 + 2), lambda a, b: oracle.dot_exact_f32(hx[a:b], hy[a:b]), n2)
    out = []
    for t in thread_counts:
        pools[t].shutdown()
        total_t = sum(b / rates[t][k] for k, b in step_bytes.items() if k in rates[t])
        total_b = sum(b for k, b in step_bytes.items() if k in rates[t])
        who = "single-thread oracle" if t == 1 else f"oracle on {t} threads (disjoint slices)"
        out.append({
            "value": round(total_b / total_t / 1e9, 3), "unit": "GB/s", "cores": t, "kind": "oracle",
            "sample": who + ": fp64 gemv N/T, two-sided gemv and ger on 16384x16384, dot on 2^28 (full size); "
                      "quantised gemv on 4096 and MX gemv on 1024 of the 16384 rows, exact dot on 2^24 "
                      "ill-conditioned pairs; "
                      "each operation's rate applied to the full step's bytes (" + "; ".join(parts[t]) + ")",
        })
    return out


def error_stats(sb, torch, ops, rows=4096, mx_rows=1024):
    """Errors of one fresh call of each step operation on the step's own
    device operands, against the CPU oracle (part of the oracle leg; the
    outputs are restored afterwards).  Per operation:
      max_err_over_bound  max over outputs of |got - oracle| / bound, with
                          the per-entry bound 2 gamma_{K+1}(u)(|c0| + sum|a||x|)
                          (binary64 u = 2^-53, binary32 2^-24);
      normwise            ||got - ref|| / ||ref||;
    GER must equal the oracle bit for bit (bitwise_equal).  The quantised and
    MX GEMVs are checked on their first `rows` / `mx_rows` rows: against the
    oracle on the decoded codes (bound as above in binary32, with |s q| <=
    1.125|a| + s 2^-9 for the row-scaled formats) and, normwise, against the
    binary64 product of the unquantised matrix.  Dot2 reports the relative
    errors of Dot2, the plain binary32 DOT and the plain binary64 DOT on the
    same pairs against the exact dot."""
    import numpy as np

    import oracle

    oracle.build()

    def g(k, u):
        return k * u / (1 - k * u)

    def h(t):
        return t.detach().cpu().numpy()

    def summarise(got, ref, bound):
        got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
        err = np.abs(got - ref)
        return {"max_err_over_bound": float((err / bound).max()), "max_abs_err": float(err.max()),
                "normwise": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))}

    res = {}
    for name, _, _, fn, ctx in ops:
        k = ctx["kind"]
        t0 = time.perf_counter()
        if k == "gemv":
            c0 = ctx["c"].clone()
            fn()
            got = h(ctx["c"])
            A, x, c0h = h(ctx["A"]), h(ctx["x"]), h(c0)
            ref = oracle.gemv(A, x, c0h, op=ctx["op"])
            mag = (np.abs(A) @ np.abs(x)) if ctx["op"] == 0 else (np.abs(x) @ np.abs(A))
            K = A.shape[1] if ctx["op"] == 0 else A.shape[0]
            res[name] = summarise(got, ref, 2 * g(K + 1, 2.0 ** -53) * (np.abs(c0h) + mag))
            ctx["c"].copy_(c0)
        elif k == "gemv2":
            c0, d0 = ctx["c"].clone(), ctx["d"].clone()
            fn()
            A, x, y = h(ctx["A"]), h(ctx["x"]), h(ctx["y"])
            rc, rd = oracle.gemv2(A, x, y, h(c0), h(d0))
            bc = 2 * g(A.shape[1] + 1, 2.0 ** -53) * (np.abs(h(c0)) + np.abs(A) @ np.abs(x))
            bd = 2 * g(A.shape[0] + 1, 2.0 ** -53) * (np.abs(h(d0)) + np.abs(y) @ np.abs(A))
            sc, sd = summarise(h(ctx["c"]), rc, bc), summarise(h(ctx["d"]), rd, bd)
            res[name] = {"c": sc, "d": sd}
            ctx["c"].copy_(c0)
            ctx["d"].copy_(d0)
        elif k == "dot":
            a0 = ctx["a"].clone()
            fn()
            x, y = h(ctx["x"]), h(ctx["y"])
            ref = oracle.dot(x, y, float(h(a0)[0]))
            bound = 2 * g(x.size + 1, 2.0 ** -53) * (abs(float(h(a0)[0])) + float(np.abs(x) @ np.abs(y)))
            got = float(h(ctx["a"])[0])
            res[name] = {"max_err_over_bound": abs(got - ref) / bound, "rel_err": abs(got - ref) / abs(ref)}
            ctx["a"].copy_(a0)
        elif k == "ger":
            C0 = ctx["C"].clone()
            fn()
            ref = oracle.ger(h(ctx["x"]), h(ctx["y"]), h(C0))
            res[name] = {"bitwise_equal": bool(np.array_equal(h(ctx["C"]).view(np.uint64), ref.view(np.uint64)))}
            ctx["C"].copy_(C0)
            del C0, ref
        elif k in ("gemv_q", "gemv_mx"):
            c0 = ctx["c"].clone()
            ctx["c"].zero_()
            fn()
            r = rows if k == "gemv_q" else mx_rows
            got = h(ctx["c"])[:r].astype(np.float64)
            x = h(ctx["x"])
            ax = np.abs(x)
            A32 = h(ctx["A"][:r]).astype(np.float32)
            if k == "gemv_q":
                bf = ctx["q"] == sb.SB_BF16
                codes = h(ctx["Q"][:r]).view(np.uint16 if bf else np.uint8)
                sc = h(ctx["s"][:r])
                oq = oracle.Q_BF16 if bf else oracle.Q_E4M3
                r1 = oracle.gemv_q(codes, sc, x, np.zeros(r), oq)
                # sum of |s q x| over the decoded codes: the codes with their sign bits cleared
                mag = oracle.gemv_q(codes & (0x7FFF if bf else 0x7F), sc, ax, np.zeros(r), oq)
            else:
                n = A32.shape[1]
                oq = oracle.Q_MXFP8 if ctx["q"] == sb.SB_MXFP8_E4M3 else oracle.Q_MXFP4
                codes = h(ctx["Q"][:r])[:, :oracle.mx_row_bytes(oq, n)]
                S = h(ctx["S"][:r])
                r1 = oracle.gemv_mx(codes, S, x, np.zeros(r), oq, n)
                mag = oracle.gemv_mx(codes & (0x7F if oq == oracle.Q_MXFP8 else 0x77), S, ax, np.zeros(r), oq, n)
            K = A32.shape[1]
            e = summarise(got, r1, 2 * g(K + 2, 2.0 ** -24) * mag)
            r2 = oracle.gemv(A32, x, np.zeros(r))
            e["normwise_vs_unquantised_f64"] = float(np.linalg.norm(got - r2) / np.linalg.norm(r2))
            e["rows"] = r
            res[name] = e
            ctx["c"].copy_(c0)
        elif k == "dot2":
            hx, hy = ctx["hx"], ctx["hy"]
            ex = oracle.dot_exact_f32(hx, hy)
            ab = oracle.dot_exact_f32(hx, hy, absval=True)
            out = {}
            a = torch.zeros(1, dtype=torch.float32, device=ctx["x"].device)
            sb.sb_dot2_f32(ctx["x"], ctx["y"], a)
            out["dot2_f32"] = float(h(a)[0])
            a = torch.zeros(1, dtype=torch.float32, device=ctx["x"].device)
            sb.sb_dot(ctx["x"], ctx["y"], a)
            out["plain_f32"] = float(h(a)[0])
            a = torch.zeros(1, dtype=torch.float64, device=ctx["x"].device)
            sb.sb_dot(ctx["x"].double(), ctx["y"].double(), a)
            out["plain_f64"] = float(h(a)[0])
            u = 2.0 ** -24
            L = 156   # longest addition path of the 2^27 launch (1024 workgroups, 128 vectors per lane)
            res[name] = {"cond": 2 * ab / abs(ex), "path_length": L,
                         "worst_case_rel_bound": (u * abs(ex) + g(L, u) ** 2 * ab) / abs(ex),
                         **{f"rel_err_{kk}": abs(v - ex) / abs(ex) for kk, v in out.items()}}
        res[name]["check_s"] = round(time.perf_counter() - t0, 2)
        log(f"errors {name}: {res[name]}")
    torch.cuda.synchronize()
    return res


def small_problems(sb, torch, dev):
    """Per-call GPU time of small problems (50 back-to-back calls replayed
    from one graph, median of 5), with the library's default cutoffs."""
    from paper_2108_02025_amd.cutoffs import per_call_us
    g = torch.Generator(device=dev)
    g.manual_seed(11)

    def uni(shape, dtype=torch.float64):
        return torch.rand(shape, generator=g, device=dev, dtype=dtype) * 2 - 1

    res = {}
    for m, n in ((1024, 1024), (150, 4096)):
        A, x, c, xt, ct = uni((m, n)), uni(n), uni(m), uni(m), uni(n)
        nb = 8 * (m * n + n + 2 * m)
        for name, fn in ((f"gemv_n_f64_{m}x{n}", lambda: sb.sb_gemv(A, x, c)),
                         (f"gemv_t_f64_{m}x{n}", lambda: sb.sb_gemv(A, xt, ct, op=1))):
            us = per_call_us(fn)
            res[name] = {"us": round(us, 2), "GB/s": round(nb / us / 1e3, 1)}
    for n in (4096, 16384, 1 << 20):
        x, y, a = uni(n), uni(n), uni(1)
        us = per_call_us(lambda: sb.sb_dot(x, y, a))
        res[f"dot_f64_{n}"] = {"us": round(us, 2), "GB/s": round(16 * n / us / 1e3, 1)}
    x, y, a = uni(16384, torch.float32), uni(16384, torch.float32), uni(1, torch.float32)
    us = per_call_us(lambda: sb.sb_dot2_f32(x, y, a))
    res["dot2_f32_16384"] = {"us": round(us, 2), "GB/s": round(8 * 16384 / us / 1e3, 1)}
    # 1024^2 binary64 GEMV-N from cold caches: a 1 GiB write (4x the
    # last-level cache and the L2s together) before every event-timed call
    m = n = 1024
    A, x, c = uni((m, n)), uni(n), uni(m)
    junk = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    ev = HipEvents(torch)
    t = []
    for _ in range(21):
        junk.fill_(0.25)
        e0 = ev.record()
        sb.sb_gemv(A, x, c)
        e1 = ev.record()
        torch.cuda.synchronize()
        t.append(1e3 * ev.ms(e0, e1))
    ev.close()
    del junk
    us = sorted(t[1:])[len(t) // 2]
    nb = 8 * (m * n + n + 2 * m)
    res["gemv_n_f64_1024x1024_cold"] = {"us": round(us, 2), "GB/s": round(nb / us / 1e3, 1),
                                        "note": "per call after a 1 GiB write, HIP events, median of 20"}
    log("small problems: " + ", ".join(f"{k} {v['us']} us" for k, v in res.items()))
    return res


def skewed_shapes(sb, torch, dev, reps=10):
    """Per-call time of the GEMVs on the skewed shapes (tall-skinny
    262144x256, short-wide 256x262144, 65536x4096 and 65537x4093 with packed
    rows) in binary64 and binary32, normal(0,1) entries: median of `reps`
    event-timed calls, each after a 2 GiB write that evicts x from the
    caches."""
    ev = HipEvents(torch)
    junk = torch.empty(1 << 28, dtype=torch.float64, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(12)
    res = {}
    for dt, es, tname in ((torch.float64, 8, "f64"), (torch.float32, 4, "f32")):
        for m, n in ((262144, 256), (256, 262144), (65536, 4096), (65537, 4093)):
            A = torch.randn((m, n), generator=g, device=dev, dtype=dt)
            for op, label, xl, cl in ((sb.SB_N, "gemv_n", n, m), (sb.SB_T, "gemv_t", m, n)):
                x = torch.randn(xl, generator=g, device=dev, dtype=dt)
                c = torch.randn(cl, generator=g, device=dev, dtype=dt)
                nb = es * (m * n + xl + 2 * cl)
                sb.sb_gemv(A, x, c, op=op)
                t = []
                for _ in range(reps):
                    junk.fill_(0.5)
                    a = ev.record()
                    sb.sb_gemv(A, x, c, op=op)
                    b = ev.record()
                    torch.cuda.synchronize()
                    t.append(1e3 * ev.ms(a, b))
                ev.close()
                us = sorted(t)[len(t) // 2]
                res[f"{label}_{tname}_{m}x{n}"] = {"us": round(us, 2), "GB/s": round(nb / us / 1e3, 1),
                                                   "frac_hbm": round(nb / us / 1e3 / PEAK_HBM_GBS, 4)}
            del A
    del junk
    log("skewed shapes: " + ", ".join(f"{k} {v['GB/s']} GB/s" for k, v in res.items()))
    return res


def host_info() -> dict:
    """The host CPU the oracle baseline ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "cpus_online": os.cpu_count(), "cpus_usable": len(os.sched_getaffinity(0))}


def device_info(torch) -> dict:
    """The GPU the step ran on: name, architecture, compute units, HBM,
    peak engine and memory clocks, and the HIP version torch was built with."""
    import ctypes
    from paper_2108_02025_amd.build import torch_lib_dir
    props = torch.cuda.get_device_properties(0)
    out = {"name": props.name, "arch": getattr(props, "gcnArchName", None),
           "compute_units": props.multi_processor_count, "hbm_bytes": props.total_memory,
           "hip": torch.version.hip}
    # hipDeviceAttribute_t values of hip_runtime_api.h (ROCm 7): peak clock
    # (kHz) 5, memory bus width (bits) 59, peak memory clock (kHz) 60
    hip = ctypes.CDLL(os.path.join(torch_lib_dir(), "libamdhip64.so"))
    for key, attr in (("clock_mhz", 5), ("memory_bus_bits", 59), ("memory_clock_mhz", 60)):
        v = ctypes.c_int(0)
        if hip.hipDeviceGetAttribute(ctypes.byref(v), attr, torch.cuda.current_device()) == 0:
            out[key] = v.value // 1000 if key.endswith("mhz") else v.value
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--ops", default=None, help="comma-separated subset of operations, in step order")
    ap.add_argument("--no-probes", action="store_true", help="skip the HBM read/copy ceiling probes")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving trace")
    ap.add_argument("--no-small", action="store_true", help="skip the small-problem latencies")
    ap.add_argument("--no-skewed", action="store_true", help="skip the skewed-shape GEMVs")
    ap.add_argument("--fenced-events", action="store_true",
                    help="time with default HIP events (system-scope release at every event)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(one process, one MI355X); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2108_02025_amd as sb
    sb.load()
    if not torch.cuda.is_available():
        sys.exit("bench.py: no GPU visible")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sel = set(args.ops.split(",")) if args.ops else None
    ops = build_ops(sb, torch, dev, sel)
    if args.ops:  # run in the order given
        order = args.ops.split(",")
        ops.sort(key=lambda o: order.index(o[0]))
    names = [o[0] for o in ops]
    log(f"ops: {names}; warmup {args.warmup}, steps {args.steps}")

    for _ in range(args.warmup):
        for _, _, _, fn, *_ in ops:
            fn()
    torch.cuda.synchronize()
    log("warmup done")

    us_per, ms_step = time_ops(torch, ops, args.steps, args.fenced_events)
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step")

    per = {}
    for name, nbytes, flops, *_ in ops:
        us = us_per[name]
        per[name] = {"us": round(us, 2), "GB/s": round(nbytes / us / 1e3, 1),
                     "frac_hbm": round(nbytes / us / 1e3 / PEAK_HBM_GBS, 4),
                     "TFLOP/s": round(flops / us / 1e6, 3), "bytes": nbytes}
    step_bytes = {name: nbytes for name, nbytes, *_ in ops}
    value = sum(step_bytes.values()) / (ms_step * 1e-3) / 1e9
    dom = max(per, key=lambda k: per[k]["us"])
    roof = {"bound": "hbm", "kernel": dom, "achieved": per[dom]["GB/s"], "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(per[dom]["GB/s"] / PEAK_HBM_GBS, 4), "traffic": measured_traffic(dom)}
    for name in per:
        t = measured_traffic(name)
        if t is not None:
            per[name]["traffic_bytes"] = t
    extras = {}
    if not args.no_probes:
        probes = build_probes(sb, torch, dev)
        for _, _, _, fn, *_ in probes:
            fn()
        p_us, _ = time_ops(torch, probes, max(3, args.steps // 2), args.fenced_events)
        ceil = {name: round(nb / p_us[name] / 1e3, 1) for name, nb, *_ in probes}
        extras["hbm_ceiling_GBs"] = {"read": ceil["probe_read"], "copy": ceil["probe_copy"],
                                     "update_ger_pattern": ceil["probe_update"]}
        for name in per:
            # GER against the read-and-rewrite probe with its own access
            # pattern; everything else against the streaming read
            ref = ceil["probe_update"] if name == "ger_f64" else ceil["probe_read"]
            per[name]["frac_ceiling"] = round(per[name]["GB/s"] / ref, 4)
        log(f"probes: read {ceil['probe_read']} GB/s, copy {ceil['probe_copy']} GB/s, "
            f"update (GER pattern) {ceil['probe_update']} GB/s")
    if all(k in per for k in ("gemv_n_f64", "gemv_t_f64", "gemv2_f64")):
        extras["gemv2_speedup_over_two_calls"] = round(
            (per["gemv_n_f64"]["us"] + per["gemv_t_f64"]["us"]) / per["gemv2_f64"]["us"], 3)
    if "gemv_n_f64" in per and "gemv_q_bf16" in per:
        extras["bf16_over_f64_flops"] = round(per["gemv_q_bf16"]["TFLOP/s"] / per["gemv_n_f64"]["TFLOP/s"], 3)
    for k, label in (("gemv_q_e4m3", "e4m3"), ("gemv_mx_fp8", "mxfp8"), ("gemv_mx_fp4", "mxfp4")):
        if "gemv_n_f64" in per and k in per:
            extras[f"{label}_over_f64_flops"] = round(per[k]["TFLOP/s"] / per["gemv_n_f64"]["TFLOP/s"], 3)

    out = {
        "metric": "GEMV HBM GB/s & % of peak, FP64 vs BF16-A; batched p50/p99 latency",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "fp64 gemv N/T and two-sided 16384x16384, dot n=2^28, ger 16384x16384; "
                               "bf16-A and e4m3-A (row scales), mxfp8-A and mxfp4-A (32-element block scales) "
                               "gemv 16384x16384 (f32 x, c); dot2 f32 n=2^27 cond 1e8",
                   "ops": names, "parallelism": "single GPU"},
        "roofline": roof, "ops": per, **extras,
    }
    if not args.no_small:
        out["small"] = small_problems(sb, torch, dev)
    if not args.no_skewed:
        out["skewed"] = skewed_shapes(sb, torch, dev)
    if not args.no_serve:
        from paper_2108_02025_amd.serve import Server, make_trace
        from paper_2108_02025_amd.tuner import TuningTable
        tuning = TuningTable.load()
        serving = {"tuned": tuning is not None}
        for label, budget, rate, dots in (("budget_4GiB", 4 << 30, 1e5, 0.0),
                                          ("budget_512MiB", 512 << 20, 1e5, 0.0),
                                          ("budget_4GiB_with_25pct_dot", 4 << 30, 1e5, 0.25),
                                          ("budget_4GiB_rate_25k", 4 << 30, 2.5e4, 0.0),
                                          ("budget_4GiB_rate_400k", 4 << 30, 4e5, 0.0)):
            trace = make_trace(4096, rate=rate, seed=501, dot_fraction=dots, dot_hi=1 << 16)
            server = Server(budget_bytes=budget, tuning=tuning, sample_every=256)  # results unchecked here
            st = server.run(trace)
            serving[label] = {"offered_rate": rate, **st.as_dict()}
            log(f"serving {label}: p50 {st.p50_ms:.2f} ms, p99 {st.p99_ms:.2f} ms, "
                f"{st.achieved_rate:.0f} req/s of {rate:.0f}, aggregate {st.aggregate_GBs:.1f} GB/s, "
                f"device-busy {st.device_busy_GBs:.1f} GB/s, {st.batches} batches, {st.rounds} rounds, "
                f"longest queue {st.max_queue}")
            del server
        out["serving"] = {"trace": "4096 requests, Poisson arrivals at offered_rate, m,n log-uniform [64,8192], "
                                   "f32 / bf16-A 50:50, uniform[-1,1), c0 = 0 (the _with_25pct_dot run "
                                   "turns a quarter of them into f32 DOTs of length log-uniform [64,65536])",
                          **serving}
    out["host"] = host_info()
    out["device"] = device_info(torch)
    if not args.no_cpu:
        log("checking every step operation against the CPU oracle")
        out["errors"] = error_stats(sb, torch, ops)
        log("timing the CPU oracle baseline")
        # The GPU machine allots 16 host threads to its one GPU, whatever the
        # machine has: the all-core figure uses at most that many.
        cores = min(16, len(os.sched_getaffinity(0)))
        res = cpu_baseline(step_bytes, (1, cores) if cores > 1 else (1,))
        out["cpu_baseline"] = res[0]
        if cores > 1:
            out["cpu_baseline_all_cores"] = {**res[1], "cap": "16 threads: the host share of one GPU on this "
                                                               "machine class"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
