"""Measurement sweeps behind the figures in profiles/ (one GPU).

    python -m paper_2108_02025_amd.measure SECTION[,SECTION...] [--reps R]

Sections (each prints one JSON line per case, times are HIP-event medians):
  batched    the batched GEMV kernel: uniform batches of bfloat16-A
             16 x 8192^2 and binary32 8 x 8192^2, the 256-request serving
             mix (tuned configurations) and its subsets by shape and kind;
             binary32 8 x 8192^2 and binary64 4 x 8192^2 as row dots
             (row-major N) and column axpys (row-major T, column-major N)
  generator  the serving loop's operand generator on 16 binary32 and 16
             bfloat16 requests of 4096^2 and on the 256-request mix
             (bytes written per second)
  narrow     the quantised and MX GEMVs (bfloat16, E4M3 row scales, MXFP8,
             MXFP4) with n = 16384 at m = 2048 .. 16384: a least-squares
             line time = fixed + bytes / marginal rate per format
  ger        GER 16384^2 binary64 beside the probes that bound it: a
             streaming read, a copy and the read-and-rewrite probe with
             GER's own access pattern
  skewed     GEMV N and T, binary64 and binary32, on 262144 x 256,
             256 x 262144, 65536 x 4096 and 65537 x 4093 beside a streaming
             read of A's bytes, each after a 2 GiB write and back to back
  serve      the serving loop: 4096 requests at 1e5/s, 4 GiB budget,
             tuned configurations (one JSON line of its statistics)
The operands are synthetic: uniform [-1, 1) and normal(0, 1) draws from
torch's seeded generator, or the serving generator's SplitMix64 streams.
"""
from __future__ import annotations

import argparse
import ctypes
import json

import numpy as np
import torch

from . import (SB_BF16, SB_FP8_E4M3, SB_MXFP4_E2M1, SB_MXFP8_E4M3, SB_N, SB_T, GemvProblem, Handle, Plan, load,
               mx_buffers, sb_gemv, sb_gemv_mx,
               sb_gemv_q, sb_ger, sb_quantize_mx, sb_quantize_rows, sb_stream_copy, sb_stream_read,
               sb_stream_update)
from .serve import GEN_DESC, device_bytes, make_trace, materialise
from .tuner import TuningTable


def timed_us(fn, reps: int) -> float:
    """Median over `reps` event-timed calls (after one untimed call)."""
    fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for k in range(reps):
        fn()
        ev[k + 1].record()
    torch.cuda.synchronize()
    t = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(reps))
    return 1e3 * t[len(t) // 2]


def emit(section: str, case: str, **kw) -> None:
    print(json.dumps({"section": section, "case": case, **kw}), flush=True)


def _requests(shapes, dev, stage, tuning, seed0=100):
    """Operands of (kind, m, n) requests materialised on the device; returns
    (buffer, problems, algorithmic bytes per problem)."""
    buf = torch.empty(sum(device_bytes(k, m, n) for k, m, n in shapes), dtype=torch.uint8, device=dev)
    off, probs, nbytes = 0, [], []
    for i, (k, m, n) in enumerate(shapes):
        probs.append(materialise(buf, off, k, m, n, seed0 + i, stage, tuning(k, m, n) if tuning else None))
        off += device_bytes(k, m, n)
        es = 4 if k == "f32" else 2
        nbytes.append(es * m * n + 4 * n + 8 * m + (4 * m if k == "bf16" else 0))
    torch.cuda.synchronize()
    return buf, probs, np.array(nbytes)


def batched(dev, reps):
    tuning = TuningTable.load()
    stage = torch.empty(8192 * 8192, dtype=torch.float32, device=dev)
    mix = [(r.kind, r.m, r.n) for r in make_trace(256, seed=501)]
    cases = [("bf16_8192x8192_x16", [("bf16", 8192, 8192)] * 16), ("f32_8192x8192_x8", [("f32", 8192, 8192)] * 8),
             ("serving_mix_256", mix)]
    for name, shapes in cases:
        buf, probs, nb = _requests(shapes, dev, stage, tuning)
        subsets = {"all": np.arange(len(shapes))}
        if name == "serving_mix_256":
            m = np.array([s[1] for s in shapes])
            n = np.array([s[2] for s in shapes])
            kind = np.array([s[0] for s in shapes])
            subsets.update({"mn_ge_2^20": np.flatnonzero(m * n >= 1 << 20), "mn_lt_2^20": np.flatnonzero(m * n < 1 << 20),
                            "n_ge_1024": np.flatnonzero(n >= 1024), "n_lt_1024": np.flatnonzero(n < 1024),
                            "f32": np.flatnonzero(kind == "f32"), "bf16": np.flatnonzero(kind == "bf16")})
        for sub, ids in subsets.items():
            plan = Plan([probs[i] for i in ids])
            us = timed_us(plan.run, reps)
            b = int(nb[ids].sum())
            emit("batched", f"{name}/{sub}", problems=len(ids), bytes=b, us=round(us, 2), GBs=round(b / us / 1e3, 1))
            del plan
        del buf, probs
    # the column-axpy form (row-major T, column-major N) beside the row dot
    # on the same 8 x 8192^2 binary32 and 4 x 8192^2 binary64 operands
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    for dt, es, count in ((torch.float32, 4, 8), (torch.float64, 8, 4)):
        As = [torch.rand((8192, 8192), generator=g, device=dev, dtype=dt) for _ in range(count)]
        xs = [torch.rand(8192, generator=g, device=dev, dtype=dt) for _ in range(count)]
        cs = [torch.zeros(8192, device=dev, dtype=dt) for _ in range(count)]
        b = count * (es * 8192 * 8192 + 3 * es * 8192)
        tname = "f32" if dt == torch.float32 else "f64"
        for label, op, view in (("rowmajor_N", SB_N, lambda A: A), ("rowmajor_T", SB_T, lambda A: A),
                                ("colmajor_N", SB_N, lambda A: A.t())):
            plan = Plan([GemvProblem(view(A), x, c, op=op) for A, x, c in zip(As, xs, cs)])
            us = timed_us(plan.run, reps)
            emit("batched", f"{tname}_8192x8192_x{count}_{label}", problems=count, bytes=b, us=round(us, 2),
                 GBs=round(b / us / 1e3, 1))
            del plan
        del As, xs, cs


def generator(dev, reps):
    L = load()
    h = Handle(dev.index)
    up = lambda v: (v + 255) // 256 * 256  # noqa: E731
    cases = [("f32_4096x4096_x16", [("f32", 4096, 4096)] * 16), ("bf16_4096x4096_x16", [("bf16", 4096, 4096)] * 16),
             ("serving_mix_256", [(r.kind, r.m, r.n) for r in make_trace(256, seed=501)])]
    for name, shapes in cases:
        buf = torch.empty(sum(device_bytes(k, m, n) for k, m, n in shapes), dtype=torch.uint8, device=dev)
        gen = np.zeros(len(shapes), dtype=GEN_DESC)
        off = written = 0
        for i, (k, m, n) in enumerate(shapes):
            es = 4 if k == "f32" else 2
            a, s_, x = up(es * m * n), up(4 * m) if k == "bf16" else 0, up(4 * n)
            base = buf.data_ptr() + off
            gen[i] = (2 if k == "bf16" else 1, 0, m, n, n, 1000 + i, base, base + a if s_ else 0, base + a + s_,
                      base + a + s_ + x)
            off += device_bytes(k, m, n)
            written += es * m * n + 4 * n + 4 * m + (4 * m if k == "bf16" else 0)
        h.prepare(int(L.sb_generate_batched_bytes(len(gen))))
        us = timed_us(lambda: h.check(L.sb_generate_batched(h.h, ctypes.c_void_p(gen.ctypes.data), len(gen))), reps)
        emit("generator", name, requests=len(shapes), bytes_written=written, us=round(us, 2),
             GBs_written=round(written / us / 1e3, 1))
        del buf


def narrow(dev, reps):
    n = 16384
    g = torch.Generator(device=dev)
    g.manual_seed(1)
    A32 = torch.rand((16384, n), generator=g, device=dev, dtype=torch.float32) * 2 - 1
    x = torch.randn(n, generator=g, device=dev, dtype=torch.float32)
    c = torch.zeros(16384, dtype=torch.float32, device=dev)
    rows = (2048, 4096, 8192, 16384)
    for fmt, q in (("bf16", SB_BF16), ("e4m3", SB_FP8_E4M3), ("mxfp8", SB_MXFP8_E4M3), ("mxfp4", SB_MXFP4_E2M1)):
        if q in (SB_BF16, SB_FP8_E4M3):
            Q = torch.empty((16384, n), dtype=torch.int16 if q == SB_BF16 else torch.uint8, device=dev)
            S = torch.empty(16384, dtype=torch.float32, device=dev)
            sb_quantize_rows(A32, Q, S, q)
            per_row = (2 if q == SB_BF16 else 1) * n + 12
            run = lambda m, Q=Q, S=S, q=q: sb_gemv_q(Q[:m], S[:m], x, c[:m], q)  # noqa: E731
        else:
            Q, S = mx_buffers(q, 16384, n, dev)
            sb_quantize_mx(A32, Q, S, q)
            per_row = (n if q == SB_MXFP8_E4M3 else n // 2) + n // 32 + 8
            run = lambda m, Q=Q, S=S, q=q: sb_gemv_mx(Q[:m], S[:m], x, c[:m], q)  # noqa: E731
        pts = []
        for m in rows:
            us = timed_us(lambda: run(m), reps)
            b = m * per_row + 4 * n
            pts.append((b, us))
            emit("narrow", f"{fmt}/{m}x{n}", bytes=b, us=round(us, 2), GBs=round(b / us / 1e3, 1))
        bb, tt = np.array(pts, dtype=float).T
        slope, fixed = np.polyfit(bb, tt, 1)
        emit("narrow", f"{fmt}/fit", fixed_us=round(float(fixed), 2), marginal_GBs=round(1e-3 / slope, 1))
        del Q, S
    del A32


def ger(dev, reps):
    M = N = 16384
    g = torch.Generator(device=dev)
    g.manual_seed(2)
    C = torch.rand((M, N), generator=g, device=dev, dtype=torch.float64)
    xs = torch.rand(M, generator=g, device=dev, dtype=torch.float64)
    ys = torch.rand(N, generator=g, device=dev, dtype=torch.float64)
    flat = C.view(-1)
    half = flat[: M * N // 2]
    dst = torch.empty_like(half)
    for name, nbytes, fn in (("ger_f64_16384x16384", 8 * (2 * M * N + M + N), lambda: sb_ger(xs, ys, C)),
                             ("update_probe_16384x16384", 2 * 8 * M * N, lambda: sb_stream_update(C)),
                             ("copy_probe_2GiB", 2 * 8 * M * N // 2, lambda: sb_stream_copy(half, dst)),
                             ("read_probe_2GiB", 8 * M * N, lambda: sb_stream_read(flat))):
        us = timed_us(fn, reps)
        emit("ger", name, bytes=nbytes, us=round(us, 2), GBs=round(nbytes / us / 1e3, 1))


def skewed(dev, reps):
    """GEMV N and T on the skewed shapes beside a streaming read of A's
    bytes: per-call times after a 2 GiB write (x, c and A out of the
    caches, as in the bench) and back to back."""
    junk = torch.empty(1 << 28, dtype=torch.float64, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(12)

    def cold_us(fn):
        fn()
        t = []
        for _ in range(reps):
            junk.fill_(0.5)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            t.append(1e3 * a.elapsed_time(b))
        return sorted(t)[len(t) // 2]

    for dt, es, tname in ((torch.float64, 8, "f64"), (torch.float32, 4, "f32")):
        for m, n in ((262144, 256), (256, 262144), (65536, 4096), (65537, 4093)):
            A = torch.randn((m, n), generator=g, device=dev, dtype=dt)
            flat = A.view(-1)[: m * n // (16 // es) * (16 // es)]  # the probe reads whole 16-byte vectors
            rb = flat.numel() * es
            rd = {"cold": cold_us(lambda: sb_stream_read(flat)), "warm": timed_us(lambda: sb_stream_read(flat), reps)}
            emit("skewed", f"read_probe_{tname}_{m}x{n}", bytes=rb,
                 **{f"{k}_us": round(v, 2) for k, v in rd.items()},
                 **{f"{k}_GBs": round(rb / v / 1e3, 1) for k, v in rd.items()})
            for op, label, xl, cl in ((SB_N, "gemv_n", n, m), (SB_T, "gemv_t", m, n)):
                x = torch.randn(xl, generator=g, device=dev, dtype=dt)
                c = torch.randn(cl, generator=g, device=dev, dtype=dt)
                nb = es * (m * n + xl + 2 * cl)
                t = {"cold": cold_us(lambda: sb_gemv(A, x, c, op=op)),
                     "warm": timed_us(lambda: sb_gemv(A, x, c, op=op), reps)}
                emit("skewed", f"{label}_{tname}_{m}x{n}", bytes=nb,
                     **{f"{k}_us": round(v, 2) for k, v in t.items()},
                     **{f"{k}_GBs": round(nb / v / 1e3, 1) for k, v in t.items()},
                     **{f"{k}_of_read_probe": round(rd[k] / t[k] * nb / rb, 3) for k in t})
            del A, flat
    del junk


def serve(dev, reps):
    """The serving loop on 4096 requests (Poisson 1e5/s, seed 501) with a
    4 GiB budget and the tuned configurations (`reps` is not used)."""
    from .serve import Server
    server = Server(budget_bytes=4 << 30, tuning=TuningTable.load(), sample_every=256)
    st = server.run(make_trace(4096, rate=1e5, seed=501))
    emit("serve", "budget_4GiB_rate_1e5", **st.as_dict())


SECTIONS = {"batched": batched, "generator": generator, "narrow": narrow, "ger": ger, "skewed": skewed,
            "serve": serve}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("sections", help="comma-separated: " + ",".join(SECTIONS))
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()
    load()
    dev = torch.device("cuda", torch.cuda.current_device())
    for s in args.sections.split(","):
        SECTIONS[s](dev, args.reps)


if __name__ == "__main__":
    main()
