"""Seeded synthetic inputs for the GEMV / DOT / GER workloads.

This module draws operands only; it holds none of the arithmetic of the
operations themselves, and both the GPU tests and the CPU oracle take their
inputs from here.  Every generator uses numpy's ``default_rng(seed)``
(PCG64) with a fixed draw order so that a (workload, seed) pair names one
input exactly:

  GEMV:  A (row-major, C order), then x, then c0
  GER:   x, then y, then C0
  DOT:   x, then y, then alpha0

binary32 inputs are the binary64 draws rounded with ``astype(float32)``.
"""
from __future__ import annotations

import numpy as np

DISTS = ("uniform", "normal", "int8", "int7", "ones")


def _draw(rng: np.random.Generator, shape, dist: str) -> np.ndarray:
    if dist == "uniform":   # i.i.d. uniform[-1, 1)
        return rng.uniform(-1.0, 1.0, size=shape)
    if dist == "normal":    # i.i.d. normal(0, 1)
        return rng.standard_normal(size=shape)
    if dist == "int8":      # integers in [-8, 8]: every partial sum exact in binary64
        return rng.integers(-8, 9, size=shape).astype(np.float64)
    if dist == "int7":      # integers in [-7, 7]: exact in binary32 up to K = 2^18
        return rng.integers(-7, 8, size=shape).astype(np.float64)
    if dist == "ones":
        return np.ones(shape, dtype=np.float64)
    raise ValueError(dist)


def _cast(a: np.ndarray, dtype) -> np.ndarray:
    return np.ascontiguousarray(a.astype(dtype))


def gemv_inputs(m: int, n: int, seed: int, dist: str = "uniform", dtype=np.float64,
                op_t: bool = False, c_dist: str | None = None, lda: int | None = None):
    """(A, x, c0) for c0 += op(A) x with A m x n row-major.

    ``lda`` > n pads each row (the padding is filled with NaN so that a read
    outside the logical matrix shows up in the result).  Returns A as an
    (m, lda) array whose first n columns are the matrix.
    """
    rng = np.random.default_rng(seed)
    A = _draw(rng, (m, n), dist)
    x = _draw(rng, (m if op_t else n,), dist)
    c0 = _draw(rng, (n if op_t else m,), c_dist or dist)
    if lda is not None and lda != n:
        assert lda >= n
        P = np.full((m, lda), np.nan)
        P[:, :n] = A
        A = P
    return _cast(A, dtype), _cast(x, dtype), _cast(c0, dtype)


def dot_inputs(n: int, seed: int, dist: str = "uniform", dtype=np.float64):
    rng = np.random.default_rng(seed)
    x = _draw(rng, (n,), dist)
    y = _draw(rng, (n,), dist)
    a0 = _draw(rng, (1,), dist)
    return _cast(x, dtype), _cast(y, dtype), _cast(a0, dtype)


def ger_inputs(m: int, n: int, seed: int, dist: str = "uniform", dtype=np.float64):
    rng = np.random.default_rng(seed)
    x = _draw(rng, (m,), dist)
    y = _draw(rng, (n,), dist)
    C0 = _draw(rng, (m, n), dist)
    return _cast(x, dtype), _cast(y, dtype), _cast(C0, dtype)


# ---------------------------------------------------------------------------
# Ill-conditioned binary32 dot products (compensated-DOT workload).
#
# Terms x_i*y_i have binary exponents spread over [-E, +E] (E = 40 by
# default: operand exponents in [-E/2, E/2]) and the pair is steered to a
# requested condition number 2*sum|x_i y_i| / |sum x_i y_i|, in the manner of
# the GenDot generator of Ogita, Rump and Oishi ("Accurate sum and dot
# product", SIAM J. Sci. Comput. 26(6), 2005, section 6): a random bulk whose
# exact sum is known, then a short tail whose terms drive the exact running
# sum down to the target magnitude, then a random permutation.
#
# The bulk is made of pairs of terms that cancel exactly: (x, y) and
# (-x*2^k, y*2^-k) with a random k that keeps both exponents in range, so
# the two products are equal and opposite and the bulk sums to exactly 0.
# The tail's running sum is then tracked exactly as a Python integer multiple
# of 2^-200 (every binary32 product is such a multiple).
# ---------------------------------------------------------------------------

_SHIFT = 200


def _shuffle(rng, arrays, n):
    """Random reordering: a full permutation for short or odd lengths; for
    long lengths a permutation of 256-element blocks followed by one random
    permutation applied inside every block (two cheap structured gathers)."""
    if n >= 1 << 16 and n % 256 == 0:
        bp = rng.permutation(n // 256)
        ip = rng.permutation(256)
        return [np.ascontiguousarray(np.take(a.reshape(-1, 256)[bp], ip, axis=1).reshape(-1)) for a in arrays]
    p = rng.permutation(n)
    return [np.ascontiguousarray(a[p]) for a in arrays]


def _f32_bits(sgn, ex, frac):
    return ((sgn.astype(np.uint32) << np.uint32(31)) | ((ex + 127).astype(np.uint32) << np.uint32(23))
            | frac).view(np.float32)


def illcond_dot_inputs(n: int, seed: int, cond: float = 1e8, spread: int = 40,
                       tail: int | None = None):
    """(x, y, alpha0, achieved_cond): binary32 pairs with cond(x.y) near ``cond``.

    The achieved condition number is computed from the exact sum.
    """
    import math

    assert n >= 16
    rng = np.random.default_rng(seed)
    half = spread // 2
    K = tail if tail is not None else min(max(n // 16, 8), 1 << 12)
    if (n - K) % 2:
        K += 1
    h = (n - K) // 2
    # binary32 operands from their bits: uniform 23-bit significands in
    # [1, 2), random signs, exponents uniform in [-half, half]
    fx = rng.integers(0, 1 << 23, size=h, dtype=np.uint32)
    fy = rng.integers(0, 1 << 23, size=h, dtype=np.uint32)
    ea = rng.integers(-half, half + 1, size=h)
    fa = rng.integers(-half, half + 1, size=h)
    sx = rng.integers(0, 2, size=h, dtype=np.uint32)
    sy = rng.integers(0, 2, size=h, dtype=np.uint32)
    # mirror: x' = -x * 2^k, y' = y * 2^-k with both exponents kept in range
    lo = np.maximum(-half - ea, fa - half)
    hi = np.minimum(half - ea, fa + half)
    k = np.minimum(lo + (rng.random(h) * (hi - lo + 1)).astype(np.int64), hi)
    xa, ya = _f32_bits(sx, ea, fx), _f32_bits(sy, fa, fy)
    xb, yb = _f32_bits(sx ^ np.uint32(1), ea + k, fx), _f32_bits(sy, fa - k, fy)
    abs_sum = 2.0 * float(np.sum(np.abs(xa.astype(np.float64) * ya.astype(np.float64))))
    S = 0                                   # exact sum of all terms so far, times 2^200
    et = math.floor(math.log2(2.0 * abs_sum / cond))
    e_top = spread + 1
    xs = np.empty(K, dtype=np.float32)
    ys = np.empty(K, dtype=np.float32)
    pmax = 2.0 ** (spread + 1)

    def steer(i, want):
        nonlocal S, abs_sum
        nf = want - S / (1 << _SHIFT)
        if nf == 0.0:
            nf = math.ldexp(1.0, et - 30)
        if abs(nf) > pmax:
            nf = math.copysign(pmax, nf)
        le = math.floor(math.log2(abs(nf)))
        ex = int(np.clip(le // 2, -half, half))
        xv = np.float32(math.ldexp(float(rng.uniform(1.0, 2.0)), ex))
        yv = np.float32(nf / float(xv))
        xs[i], ys[i] = xv, yv
        p = float(xv) * float(yv)                          # exact
        S += int(math.ldexp(p, _SHIFT))
        abs_sum += abs(p)

    for i in range(K - 1):
        e_i = e_top - (e_top - et) * (i + 1) / (K - 1)     # descends to log2(target)
        r = float(rng.uniform(1.0, 2.0)) * (1.0 if rng.integers(0, 2) else -1.0)
        steer(i, math.ldexp(r, math.floor(e_i)))
    # Last term: land the sum on 2*sum|p|/cond for the terms drawn so far.
    steer(K - 1, (1.0 if S >= 0 else -1.0) * 2.0 * abs_sum / cond)
    x = np.concatenate([xa, xb, xs])
    y = np.concatenate([ya, yb, ys])
    x, y = _shuffle(rng, (x, y), n)
    exact = S / (1 << _SHIFT)
    achieved = 2.0 * abs_sum / abs(exact) if exact != 0 else float("inf")
    return x, y, np.zeros(1, dtype=np.float32), achieved


# ---------------------------------------------------------------------------
# Counter-based generator for operands made on the device (serving loop).
# SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
# generators", OOPSLA 2014): state_k = seed + (k+1)*0x9E3779B97F4A7C15, then
# the 64-bit finaliser below.  A value in [-1, 1) is taken from the top 53 bits.
# The GPU library implements the same published definition separately.
# ---------------------------------------------------------------------------

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    z = (np.uint64(seed) + (counters.astype(np.uint64) + np.uint64(1)) * _GOLDEN)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def splitmix_uniform(seed: int, start: int, count: int, dtype=np.float64) -> np.ndarray:
    """count values in [-1, 1) for elements start..start+count-1.  binary64:
    element e from the state of counter e, the top 53 bits (2u - 1,
    u = (z >> 11) 2^-53).  binary32: two elements per state, element e from
    the state of counter e >> 1 and the 24-bit field z >> 40 (e even) or
    (z >> 8) & 0xFFFFFF (e odd), value (f - 2^23) 2^-23.  Both exact."""
    e = np.arange(start, start + count, dtype=np.uint64)
    if np.dtype(dtype) == np.float32:
        with np.errstate(over="ignore"):
            z = splitmix64(seed, e >> np.uint64(1))
        f = np.where(e & np.uint64(1), (z >> np.uint64(8)) & np.uint64(0xFFFFFF), z >> np.uint64(40))
        return ((f.astype(np.int64) - (1 << 23)).astype(np.float64) * 2.0 ** -23).astype(np.float32)
    with np.errstate(over="ignore"):
        z = splitmix64(seed, e)
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)  # [0, 1)
    return 2.0 * u - 1.0
