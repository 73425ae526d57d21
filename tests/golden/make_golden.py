"""Writes the small text fixtures in this folder.  It calls only the CPU
oracle (and the seeded input generators); no value here comes from the GPU.

  gemv_small.txt  GEMV (section 3.1 definition, Algorithms 1 and 2): a 5 x 7
                  integer example, all four (layout, op) pairs
  dot_small.txt   DOT (section 3.1 definition, Algorithms 3 and 4)
  ger_small.txt   GER / GEM (section 3.1 definition, Algorithm 2)
  e4m3fn_codes.txt  value of every OCP E4M3FN code (precision form storage)

Run:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def fmt(v):
    return " ".join(float(t).hex() for t in np.ravel(v))


def main():
    m, n = 5, 7
    A = (np.arange(m * n).reshape(m, n) % 11 - 5).astype(np.float64)
    xn = (np.arange(n) % 5 - 2).astype(np.float64)
    xt = (np.arange(m) % 3 - 1).astype(np.float64)
    cn = np.arange(m, dtype=np.float64) - 2
    ct = np.arange(n, dtype=np.float64) * 0.5
    with open(os.path.join(HERE, "gemv_small.txt"), "w") as f:
        f.write("# GEMV c += op(A) x; A is 5x7 with A[i][j] = (7i+j) mod 11 - 5 (row-major)\n")
        f.write("# lines: name then hex floats; 'A' row-major, 'xN','cN0','cN' for op N, 'xT','cT0','cT' for op T\n")
        f.write("A " + fmt(A) + "\n")
        f.write("xN " + fmt(xn) + "\ncN0 " + fmt(cn) + "\n")
        f.write("cN " + fmt(oracle.gemv(A, xn, cn, op=oracle.OP_N)) + "\n")
        f.write("xT " + fmt(xt) + "\ncT0 " + fmt(ct) + "\n")
        f.write("cT " + fmt(oracle.gemv(A, xt, ct, op=oracle.OP_T)) + "\n")
    x = np.array([0.5, -1.25, 3.0, 2.0 ** -20, -7.0])
    y = np.array([4.0, 0.75, -1.5, 2.0 ** 20, 0.125])
    with open(os.path.join(HERE, "dot_small.txt"), "w") as f:
        f.write("# DOT alpha += x . y\n")
        f.write("x " + fmt(x) + "\ny " + fmt(y) + "\nalpha0 " + fmt([10.0]) + "\n")
        f.write("alpha " + fmt([oracle.dot(x, y, 10.0)]) + "\n")
    gx = np.array([1.0, -2.0, 0.5])
    gy = np.array([3.0, 0.25, -4.0, 8.0])
    C0 = np.arange(12, dtype=np.float64).reshape(3, 4)
    with open(os.path.join(HERE, "ger_small.txt"), "w") as f:
        f.write("# GER C += x (outer) y, C 3x4 row-major\n")
        f.write("x " + fmt(gx) + "\ny " + fmt(gy) + "\nC0 " + fmt(C0) + "\n")
        f.write("C " + fmt(oracle.ger(gx, gy, C0)) + "\n")
    with open(os.path.join(HERE, "e4m3fn_codes.txt"), "w") as f:
        f.write("# OCP 8-bit floating point E4M3FN: code (hex) and value; NaN for S.1111.111\n")
        for c in range(256):
            v = oracle.e4m3_to_f32(c)
            f.write("%02x %s\n" % (c, "nan" if v != v else float(v).hex()))


if __name__ == "__main__":
    main()
