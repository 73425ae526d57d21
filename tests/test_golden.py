"""The stored fixtures agree with exact arithmetic and with the oracle."""
from fractions import Fraction

import numpy as np

import goldens


def test_gemv_golden(orc):
    g = goldens.load("gemv_small.txt")
    A = g["A"].reshape(5, 7)
    ai = A.astype(np.int64)
    assert np.array_equal(g["cN"], g["cN0"] + ai @ g["xN"].astype(np.int64))
    assert np.array_equal(g["cT"], g["cT0"] + ai.T @ g["xT"].astype(np.int64))
    assert np.array_equal(orc.gemv(A, g["xN"], g["cN0"]), g["cN"])
    assert np.array_equal(orc.gemv(A, g["xT"], g["cT0"], op=1), g["cT"])


def test_dot_golden(orc):
    g = goldens.load("dot_small.txt")
    exact = Fraction(g["alpha0"][0]) + sum(Fraction(a) * Fraction(b) for a, b in zip(g["x"], g["y"]))
    assert g["alpha"][0] == float(exact)  # every partial sum here is exact
    assert orc.dot(g["x"], g["y"], g["alpha0"][0]) == g["alpha"][0]


def test_ger_golden(orc):
    g = goldens.load("ger_small.txt")
    C = g["C0"].reshape(3, 4) + np.outer(g["x"], g["y"])
    assert np.array_equal(g["C"].reshape(3, 4), C)
    assert np.array_equal(orc.ger(g["x"], g["y"], g["C0"].reshape(3, 4)), C)


def test_e4m3_golden_table():
    t = goldens.e4m3_table()
    assert len(t) == 256
    for code, v in t.items():
        E, M = (code >> 3) & 15, code & 7
        if E == 15 and M == 7:
            assert v != v
            continue
        mag = Fraction(M, 512) if E == 0 else Fraction(8 + M, 8) * Fraction(2) ** (E - 7)
        assert Fraction(v) == (-mag if code & 0x80 else mag)
