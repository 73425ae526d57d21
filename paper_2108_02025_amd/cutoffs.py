"""Measure the small-problem cutoffs on the current GPU.

Section 4.3 of the paper picks its small-problem dot product below a size
found by experiment; this tool does that experiment for the library's two
single-launch forms by timing each size with the form forced on and forced
off through the handle's cutoffs (``sb_set_cutoff``):

  * DOT, binary32 DOT and Dot2: one workgroup that also adds alpha, against
    the two-stage reduction, for n = 2^8 .. 2^22;
  * column-axpy GEMV (row-major c += A^T x): unsplit with 16 waves per
    column block, against the row split, for rows 64 .. 1024 and columns
    128 .. 16384.

Each time is the per-call GPU time of 50 back-to-back calls captured in one
graph (median of 5 replays), so launch gaps are counted as a caller that
issues many small calls sees them.  The report gives both times per size
and the cutoff values they imply (the largest size below which the
single-launch form is faster at every measured point).

    python -m paper_2108_02025_amd.cutoffs [--out FILE]
"""
from __future__ import annotations

import argparse
import math

import torch

from . import (SB_CUTOFF_DOT_SMALL_BYTES, SB_CUTOFF_GEMV_T_SMALL_SPLITS, handle_for, sb_dot, sb_dot2_f32,
               sb_gemv, sb_get_cutoff, sb_set_cutoff)

FORCE_ON, FORCE_OFF = 1 << 62, 0
CALLS, REPS = 50, 5


def per_call_us(fn, calls: int = CALLS, reps: int = REPS) -> float:
    """Median per-call GPU time of `calls` back-to-back calls of fn replayed
    from one captured graph."""
    fn()  # sizes the workspace before capture
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        fn()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            for _ in range(calls):
                fn()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        a.record()
        g.replay()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b) * 1e3 / calls)
    return sorted(ts)[reps // 2]


def _pair(which: int, fn, handle) -> tuple[float, float]:
    keep = sb_get_cutoff(which, handle)
    try:
        sb_set_cutoff(which, FORCE_ON, handle)
        on = per_call_us(fn)
        sb_set_cutoff(which, FORCE_OFF, handle)
        off = per_call_us(fn)
    finally:
        sb_set_cutoff(which, keep, handle)
    return on, off


def measure_dot(device, log=print) -> dict:
    out = {}
    for kind, dt in (("dot_f64", torch.float64), ("dot_f32", torch.float32), ("dot2_f32", torch.float32)):
        rows = []
        for e in range(8, 23):
            n = 1 << e
            x = torch.rand(n, device=device, dtype=dt)
            y = torch.rand(n, device=device, dtype=dt)
            al = torch.zeros(1, device=device, dtype=dt)
            fn = (lambda: sb_dot2_f32(x, y, al)) if kind == "dot2_f32" else (lambda: sb_dot(x, y, al))
            on, off = _pair(SB_CUTOFF_DOT_SMALL_BYTES, fn, handle_for(x))
            rows.append({"n": n, "bytes": 2 * n * x.element_size(), "single_us": round(on, 2),
                         "two_stage_us": round(off, 2)})
            log(f"{kind} n={n}: single workgroup {on:.2f} us, two-stage {off:.2f} us")
        out[kind] = rows
    return out


def measure_gemv_t(device, log=print) -> dict:
    out = {}
    for kind, dt in (("gemv_t_f64", torch.float64), ("gemv_t_f32", torch.float32)):
        rows = []
        for r in (128, 192, 256, 384, 512, 1024):
            for c in (128, 1024, 4096, 16384):
                A = torch.rand((r, c), device=device, dtype=dt)
                x = torch.rand(r, device=device, dtype=dt)
                cv = torch.zeros(c, device=device, dtype=dt)
                on, off = _pair(SB_CUTOFF_GEMV_T_SMALL_SPLITS, lambda: sb_gemv(A, x, cv, op=1), handle_for(A))
                rows.append({"rows": r, "cols": c, "splits": _splits(r, c, A.element_size()),
                             "unsplit_us": round(on, 2), "split_us": round(off, 2)})
                log(f"{kind} {r}x{c}: unsplit {on:.2f} us, split {off:.2f} us")
        out[kind] = rows
    return out


def _splits(rows: int, cols: int, esize: int) -> int:
    """Ways of the row split the column-axpy plan would use (its rule:
    about 1024 workgroups, at most 512 ways, at least 64 rows per part)."""
    ncb = max(1, -(-cols // (64 * 16 // esize)))
    ns = max(1, min(-(-1024 // ncb), 512, rows // 64))
    rs = -(-rows // ns)
    return -(-rows // rs)


def recommend(res: dict) -> dict:
    """Cutoffs implied by the measurements."""
    dot_bytes = math.inf
    for rows in (res[k] for k in ("dot_f64", "dot_f32", "dot2_f32")):
        best = 0
        for r in rows:
            if r["single_us"] < r["two_stage_us"]:
                best = r["bytes"]
            else:
                break
        dot_bytes = min(dot_bytes, best)
    splits = None
    by_ns = {}
    for k in ("gemv_t_f64", "gemv_t_f32"):
        for r in res[k]:
            by_ns.setdefault(r["splits"], []).append(r["unsplit_us"] < r["split_us"])
    splits = 0
    for ns in sorted(by_ns):
        if ns < 2:
            continue
        if all(by_ns[ns]):
            splits = ns
        else:
            break
    return {"dot_small_bytes": int(dot_bytes), "gemv_t_small_splits": int(splits)}


def report(res: dict, rec: dict) -> str:
    lines = ["| operation | n | operand bytes | single workgroup us | two-stage us |", "|---|---|---|---|---|"]
    for k in ("dot_f64", "dot_f32", "dot2_f32"):
        for r in res[k]:
            lines.append(f"| {k} | {r['n']} | {r['bytes']} | {r['single_us']} | {r['two_stage_us']} |")
    lines += ["", "| operation | rows x cols | row split (ways) | unsplit us | split us |", "|---|---|---|---|---|"]
    for k in ("gemv_t_f64", "gemv_t_f32"):
        for r in res[k]:
            lines.append(f"| {k} | {r['rows']} x {r['cols']} | {r['splits']} | {r['unsplit_us']} | {r['split_us']} |")
    lines += ["", f"implied cutoffs: SB_CUTOFF_DOT_SMALL_BYTES = {rec['dot_small_bytes']}, "
                  f"SB_CUTOFF_GEMV_T_SMALL_SPLITS = {rec['gemv_t_small_splits']}",
              f"library defaults: SB_CUTOFF_DOT_SMALL_BYTES = {sb_get_cutoff(SB_CUTOFF_DOT_SMALL_BYTES)}, "
              f"SB_CUTOFF_GEMV_T_SMALL_SPLITS = {sb_get_cutoff(SB_CUTOFF_GEMV_T_SMALL_SPLITS)}"]
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", help="write the markdown report here")
    args = ap.parse_args()
    dev = torch.device("cuda", torch.cuda.current_device())
    torch.manual_seed(0)
    res = {**measure_dot(dev), **measure_gemv_t(dev)}
    text = report(res, recommend(res))
    print(text)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")


if __name__ == "__main__":
    main()
