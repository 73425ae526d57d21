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
# product", SIAM J. Sci. Comput. 26(6), 2005, section 6): a random bulk,
# then a tail whose terms drive the exact running sum down to the target
# magnitude, then a random permutation.  The running sum is kept exactly as a
# Python integer multiple of 2^-SHIFT.
# ---------------------------------------------------------------------------

_SHIFT = 200  # every binary32 product used here is a multiple of 2^-200


def exact_sum_scaled(p: np.ndarray) -> int:
    """Exact sum of binary64 values that are multiples of 2^-200 with
    magnitude below 2^64, returned as the integer (sum * 2^200).

    Positive and negative terms are handled apart; each magnitude is scaled
    to an integer-valued binary64 and split into 52-bit limbs with exact
    floor/subtract steps (the remainder is a subset of the value's bits), and
    each limb column is summed in int64 blocks that cannot overflow.
    """
    p = np.asarray(p, dtype=np.float64)
    total = 0
    for sgn, sel in ((1, p > 0), (-1, p < 0)):
        rem = np.ldexp(np.abs(p[sel]), _SHIFT)
        assert np.all(rem < 2.0 ** 264), "term too large"
        part = 0
        for k in (260, 208, 156, 104, 52, 0):
            q = np.floor(np.ldexp(rem, -k))
            rem = rem - np.ldexp(q, k)
            qi = q.astype(np.int64)          # each limb is below 2^52
            acc = 0
            for s0 in range(0, qi.shape[0], 1 << 10):
                acc += int(qi[s0:s0 + (1 << 10)].sum())
            part += acc << k
        assert not np.any(rem), "term not a multiple of 2^-200"
        total += sgn * part
    return total


def illcond_dot_inputs(n: int, seed: int, cond: float = 1e8, spread: int = 40,
                       tail: int | None = None):
    """(x, y, alpha0, achieved_cond): binary32 pairs with cond(x.y) near ``cond``.

    The achieved condition number is measured from the exact sum.
    """
    import math

    assert n >= 16
    rng = np.random.default_rng(seed)
    half = spread // 2
    K = tail if tail is not None else min(max(n // 16, 8), 1 << 12)
    n1 = n - K

    def rand_f32(size, emin, emax):
        mant = rng.uniform(1.0, 2.0, size=size)
        ex = rng.integers(emin, emax + 1, size=size)
        sgn = np.where(rng.integers(0, 2, size=size) == 1, -1.0, 1.0)
        return (sgn * np.ldexp(mant, ex)).astype(np.float32)

    x1 = rand_f32(n1, -half, half)
    y1 = rand_f32(n1, -half, half)
    p1 = x1.astype(np.float64) * y1.astype(np.float64)   # exact products
    S = exact_sum_scaled(p1)                              # sum * 2^200, exact
    abs_sum = float(np.sum(np.abs(p1)))
    et = math.floor(math.log2(2.0 * abs_sum / cond))
    xs = np.empty(K, dtype=np.float32)
    ys = np.empty(K, dtype=np.float32)
    pmax = 2.0 ** (spread + 1)

    def steer(k, want):
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
        xs[k], ys[k] = xv, yv
        p = float(xv) * float(yv)                          # exact
        S += int(math.ldexp(p, _SHIFT))
        abs_sum += abs(p)

    for k in range(K - 1):
        e_k = spread - (spread - et) * (k + 1) / (K - 1)   # descends to log2(target)
        r = float(rng.uniform(1.0, 2.0)) * (1.0 if rng.integers(0, 2) else -1.0)
        steer(k, math.ldexp(r, math.floor(e_k)))
    # Last term: land the sum on 2*sum|p|/cond for the terms drawn so far.
    sign = 1.0 if S >= 0 else -1.0
    steer(K - 1, sign * 2.0 * abs_sum / cond)
    x = np.concatenate([x1, xs])
    y = np.concatenate([y1, ys])
    perm = rng.permutation(n)
    x, y = np.ascontiguousarray(x[perm]), np.ascontiguousarray(y[perm])
    abs_all = float(np.sum(np.abs(x.astype(np.float64) * y.astype(np.float64))))
    exact = S / (1 << _SHIFT)
    achieved = 2.0 * abs_all / abs(exact) if exact != 0 else float("inf")
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


def splitmix_uniform(seed: int, start: int, count: int) -> np.ndarray:
    """count values in [-1, 1) (binary64) from counters start..start+count-1."""
    with np.errstate(over="ignore"):
        z = splitmix64(seed, np.arange(start, start + count, dtype=np.uint64))
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)  # [0, 1)
    return 2.0 * u - 1.0
