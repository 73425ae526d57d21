"""The reduction tree of the library's compensated binary32 DOT, stated for
the tests: which workgroup, wave, lane, vector component and loop iteration
reads element e, and the longest chain of additions any product passes
through.  The tests use it to place a few large, cancelling products so that
they meet first at one chosen merge level (a level-isolating check), and to
evaluate the Ogita-Rump-Oishi error bound with the real path length.

The tree (workgroups of NT threads, 16-byte loads, four binary32 lanes per
vector component q):
  large problems (x and y above the single-workgroup cutoff): G workgroups
    own contiguous chunks of `chunk` elements; thread t of workgroup b reads
    vector v = t + NT*k (k = 0, 1, ...) of its chunk, i.e. elements
    b*chunk + 4*v + q, folding them into one (sum, error) pair per q in
    increasing k; the four pairs merge in q order; a 64-lane butterfly
    (xor 32, 16, 8, 4, 2, 1) merges a wave; thread 0 merges the waves'
    pairs in wave order and writes the workgroup's pair; a second kernel
    of 256 threads merges partials i, i + 256, ... per thread, then the
    same butterfly and wave order, and adds alpha last.
  small problems: one workgroup of 1024 threads does the first part over
    the whole vector and adds alpha itself.
Unaligned operands (a base not on a 16-byte boundary) read one element per
thread (q = 0 only).
"""
from __future__ import annotations

import math

SMALL_BYTES = 256 * 1024   # default single-workgroup cutoff (x and y bytes)
MAX_BLOCKS = 1024
UNROLL = 16
WAVE = 64


def ceil_div(a: int, b: int) -> int:
    return -(-a // b)


def plan(n: int, small_bytes: int = SMALL_BYTES) -> dict:
    """Launch shape of the compensated DOT for n binary32 pairs."""
    if n * 8 <= small_bytes:
        return {"small": True, "NT": 1024, "nblocks": 1, "chunk": n}
    nt = 256
    step = nt * 4
    nb = max(1, min(ceil_div(n, step * UNROLL), MAX_BLOCKS))
    chunk = ceil_div(ceil_div(n, nb), step) * step
    return {"small": False, "NT": nt, "nblocks": max(1, ceil_div(n, chunk)), "chunk": chunk}


def element(p: dict, b: int = 0, w: int = 0, lane: int = 0, q: int = 0, k: int = 0,
            aligned: bool = True) -> int:
    """Index of the element that workgroup b, wave w, lane `lane` reads as
    component q of its k-th vector (aligned) or its k-th element (unaligned)."""
    t = w * WAVE + lane
    if aligned:
        return b * p["chunk"] + 4 * (t + p["NT"] * k) + q
    return b * p["chunk"] + t + p["NT"] * k


def path_length(n: int, small_bytes: int = SMALL_BYTES) -> int:
    """Longest chain of floating-point additions from a product to the
    result: the lane's chain, the merge of the four components, the
    butterfly, the waves in order, then (large problems) the second stage's
    per-thread chain, butterfly and waves, and alpha with its final sum."""
    p = plan(n, small_bytes)
    nt = p["NT"]
    chain = ceil_div(p["chunk"], 4 * nt) + 1          # vectors per lane, plus a scalar tail
    first = chain + 3 + int(math.log2(WAVE)) + (nt // WAVE - 1)
    if p["small"]:
        return first + 2
    second = ceil_div(p["nblocks"], 256) + int(math.log2(WAVE)) + (256 // WAVE - 1)
    return first + second + 2
