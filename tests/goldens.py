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


def load_hex(name):
    """Fixture of hexadecimal integers (bit patterns): key -> int64 array."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            out[key] = np.array([int(v, 16) for v in vals], dtype=np.int64)
    return out


def quantize_special_rows():
    """The rows of quantize_special_rows.txt as a binary32 matrix, and per
    format ("bf16", "e4m3") the expected scale bits and codes."""
    d = load_hex("quantize_special_rows.txt")
    k = sorted(int(key[3:]) for key in d if key.startswith("row"))
    rows = np.stack([d[f"row{i}"].astype(np.uint32) for i in k]).view(np.float32)
    exp = {}
    for fmt, ct in (("bf16", np.uint16), ("e4m3", np.uint8)):
        s = np.array([d[f"{fmt}_s{i}"][0] for i in k], dtype=np.uint32)
        q = np.stack([d[f"{fmt}_q{i}"].astype(ct) for i in k])
        exp[fmt] = (s, q)
    return rows, exp
