"""Autotuner for the batched GEMV kernel.

For every bucket (kind, round(log2 m), round(log2 n)) with kind binary64,
binary32, bfloat16-A or E4M3-A and m, n in [64, 8192], the tuner builds a
batch of identical problems of the bucket's shape (operands made on the
device), times each candidate configuration

    group          lanes per row (rows per wave = 64 / group): the powers of
                   two 4..64 that leave each lane at least one 16-byte load
    split          column chunks (tile width n / split; split-K): the fewest
                   whose x chunk fits 32 KiB of LDS (the kernel takes up to
                   64 KiB; the table was measured with 32), plus twice and
                   four times that for short, wide shapes
    rows_per_tile  tile height: automatic (about 256 KiB of A, at most eight
                   row passes), or two or sixteen row passes of the workgroup

with HIP events (median of several launches over the same table) and keeps
the fastest.  Waves per workgroup, loads in flight per lane and the grid are
fixed when the library is built (measured: two 4-wave workgroups per
compute unit with 8 loads in flight for binary64, binary32 and bfloat16
codes and 4 for E4M3; as build-time constants they cost no registers).  The
table is saved as JSON keyed by GPU architecture and library version;
`TuningTable` maps any (kind, m, n) to its bucket's configuration.  A
problem's configuration depends only on its own shape, so tuning never
breaks the alone-vs-mix equality of results.

    python -m paper_2108_02025_amd.tuner [--out FILE] [--quick]
"""
from __future__ import annotations

import argparse
import json
import math
import os

import numpy as np
import torch

from . import (SB_BF16, SB_FP8_E4M3, BatchTable, GemvProblem, StreamBlasError, sb_gemv_batched_table_bytes,
               sb_quantize_rows, sb_version)
from .serve import GEN_DESC, device_bytes

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning_gfx950.json")
LOG2 = range(6, 14)  # 64 .. 8192


def bucket(kind: str, m: int, n: int) -> str:
    lm = min(max(int(round(math.log2(max(m, 1)))), LOG2[0]), LOG2[-1])
    ln = min(max(int(round(math.log2(max(n, 1)))), LOG2[0]), LOG2[-1])
    return f"{kind}/{lm}/{ln}"


ESIZE = {"f64": 8, "f32": 4, "bf16": 2, "e4m3": 1}   # bytes per element of A


def candidates(kind: str, m: int, n: int) -> list[dict]:
    per16 = 16 // ESIZE[kind]                  # elements per 16-byte load
    out = []
    for g in (4, 8, 16, 32, 64):
        if g > 4 and (n + per16 - 1) // per16 < g:
            continue
        s0 = max(1, -(-n * (8 if kind == "f64" else 4) // 32768))   # x chunks must fit 32 KiB of LDS
        splits = [s0]
        if n >= 2048 and m <= 1024:
            splits += [2 * s0, 4 * s0]
        rpass = 4 * (64 // g)                  # rows of one pass of a 4-wave workgroup
        heights = [0] + [h for h in (2 * rpass, 16 * rpass) if h < m]
        for sp in splits:
            for rt in heights:
                out.append({"group": g, "rows_per_tile": rt, "split": sp})
    return out


def problem_bytes(kind: str, m: int, n: int) -> int:
    return ESIZE[kind] * m * n


def _make_batch(kind: str, m: int, n: int, count: int, device):
    """`count` problems of one shape with operands made on the device:
    binary32 and bfloat16-A by the serving loop's generator, binary64 and
    E4M3-A from torch's seeded uniform draws (E4M3 quantised per row)."""
    from . import Handle, load
    if kind in ("f64", "e4m3"):
        g = torch.Generator(device=device)
        g.manual_seed(777)
        dt = torch.float64 if kind == "f64" else torch.float32
        views = []
        for _ in range(count):
            A = torch.rand((m, n), generator=g, device=device, dtype=dt) * 2 - 1
            sc = None
            if kind == "e4m3":
                Aq = torch.empty((m, n), dtype=torch.uint8, device=device)
                sc = torch.empty(m, dtype=torch.float32, device=device)
                sb_quantize_rows(A, Aq, sc, SB_FP8_E4M3)
                A = Aq
            xv = torch.rand(n, generator=g, device=device, dtype=dt) * 2 - 1
            views.append((A, sc, xv, torch.zeros(m, dtype=dt, device=device)))
        return None, views
    per = device_bytes(kind, m, n)
    buf = torch.empty(per * count, dtype=torch.uint8, device=device)
    base = buf.data_ptr()
    es = 4 if kind == "f32" else 2
    up = lambda v: (v + 255) // 256 * 256  # noqa: E731
    a, s_, x = up(es * m * n), up(4 * m) if kind == "bf16" else 0, up(4 * n)
    gen = np.zeros(count, dtype=GEN_DESC)
    offs = base + per * np.arange(count, dtype=np.uint64)
    gen["dtype"] = 2 if kind == "bf16" else 1
    gen["m"], gen["n"], gen["lda"], gen["seed"] = m, n, n, 777 + np.arange(count)
    gen["A"], gen["x"], gen["c"] = offs, offs + a + s_, offs + a + s_ + x
    gen["scales"] = offs + a if kind == "bf16" else 0
    L = load()
    h = Handle(device.index)
    h.prepare(int(L.sb_generate_batched_bytes(count)))
    import ctypes
    h.check(L.sb_generate_batched(h.h, ctypes.c_void_p(gen.ctypes.data), count))
    views = []
    for k in range(count):
        o = per * k
        A = buf[o:o + es * m * n].view(torch.float32 if kind == "f32" else torch.int16).view(m, n)
        sc = buf[o + a:o + a + 4 * m].view(torch.float32) if kind == "bf16" else None
        xv = buf[o + a + s_:o + a + s_ + 4 * n].view(torch.float32)
        cv = buf[o + a + s_ + x:o + a + s_ + x + 4 * m].view(torch.float32)
        views.append((A, sc, xv, cv))
    return buf, views


def time_config(kind, m, n, cfg, views, table: BatchTable, reps=7) -> float:
    q = {"bf16": SB_BF16, "e4m3": SB_FP8_E4M3}.get(kind)
    probs = [GemvProblem(A, xv, cv, scales=sc, q=q, **cfg) for A, sc, xv, cv in views]
    try:
        if sb_gemv_batched_table_bytes(probs)[0] > table.capacity:
            return math.inf
    except StreamBlasError:
        return math.inf   # not a valid configuration for this shape (e.g. x chunk above 32 KiB)
    table.encode(probs)
    table.run()
    evs = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        table.run()
        b.record()
        evs.append((a, b))
    torch.cuda.synchronize()
    return sorted(x.elapsed_time(y) for x, y in evs)[reps // 2] * 1e3


def tune(kinds=("f32", "bf16", "f64", "e4m3"), buckets=None, batch_bytes=96 << 20, max_count=64,
         log=print) -> dict:
    dev = torch.device("cuda", torch.cuda.current_device())
    bt = BatchTable(64 << 20, dev)
    table = {}
    for kind in kinds:
        for lm in LOG2:
            for ln in LOG2:
                key = f"{kind}/{lm}/{ln}"
                if buckets and key not in buckets:
                    continue
                m, n = 1 << lm, 1 << ln
                count = max(1, min(max_count, batch_bytes // problem_bytes(kind, m, n)))
                buf, views = _make_batch(kind, m, n, count, dev)
                best = None
                for cfg in candidates(kind, m, n):
                    us = time_config(kind, m, n, cfg, views, bt)
                    if best is None or us < best[0]:
                        best = (us, cfg)
                auto_us = time_config(kind, m, n, {"group": 0, "rows_per_tile": 0, "split": 0}, views, bt)
                gbs = count * problem_bytes(kind, m, n) / best[0] / 1e3
                table[key] = {**best[1], "us": round(best[0], 2), "auto_us": round(auto_us, 2),
                              "GBs": round(gbs, 1), "count": int(count)}
                log(f"{key}: {best[1]} {best[0]:.1f} us (automatic {auto_us:.1f} us), {gbs:.0f} GB/s")
                del buf, views
    return {"arch": "gfx950", "library_version": sb_version(), "buckets": table}


class TuningTable:
    """Callable (kind, m, n) -> configuration dict, from a saved table."""

    def __init__(self, data: dict):
        self.buckets = data["buckets"]

    @classmethod
    def load(cls, path: str = DEFAULT_TABLE) -> "TuningTable | None":
        if not os.path.exists(path):
            return None
        with open(path) as f:
            data = json.load(f)
        if data.get("arch") != "gfx950" or data.get("library_version") != sb_version():
            return None
        return cls(data)

    def __call__(self, kind: str, m: int, n: int) -> dict | None:
        if n > 1 << LOG2[-1]:
            return None  # beyond the tuned widths: the automatic split fits any row
        e = self.buckets.get(bucket(kind, m, n))
        if e is None:
            return None
        # a bucket spans widths up to 2^0.5 times its centre: raise the split
        # where this width's x chunk would not fit 32 KiB of LDS
        xs = 8 if kind == "f64" else 4
        split = e["split"]
        while split and -(-n // split) * xs > 32768:
            split += 1
        return {"group": e["group"], "rows_per_tile": e["rows_per_tile"], "split": split}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--quick", action="store_true", help="tune a few buckets only")
    args = ap.parse_args()
    buckets = None
    if args.quick:
        buckets = {"f32/13/13", "bf16/13/13", "f32/6/13", "bf16/13/6", "f32/10/10", "f64/12/12", "e4m3/10/13"}
    data = tune(buckets=buckets)
    with open(args.out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(f"wrote {args.out} ({len(data['buckets'])} buckets)")


if __name__ == "__main__":
    main()
