"""Reader for the text fixtures under tests/golden/ (written by
tests/golden/make_golden.py from the CPU oracle only)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            out[key] = np.array([float.fromhex(v) for v in vals])
    return out


def e4m3_table():
    vals = {}
    with open(os.path.join(GOLDEN, "e4m3fn_codes.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            code, v = line.split()
            vals[int(code, 16)] = float("nan") if v == "nan" else float.fromhex(v)
    return vals
