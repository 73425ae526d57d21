"""Level-isolating checks of the compensated binary32 DOT (Dot2: TwoProduct
and TwoSum at every step and every merge level, Ogita, Rump and Oishi 2005).

Each case places three non-zero products in otherwise zero vectors: +2^40,
1 and -2^40, positioned (from the tree in tests/dot2_tree.py) so that +2^40
and 1 first meet at one chosen level of the reduction and -2^40 joins only
at a later level.  The exact dot product is 1.  A level that merges its
(sum, error) pairs with TwoSum keeps the 1 in the error term and the result
is exactly 1; a level that adds plainly rounds 2^40 + 1 to 2^40 and the
result is 0.  So every case pins one level, and the plain binary32 DOT on
the same vectors (which loses the 1) shows that the case has teeth.  The
expected value is the exact long-accumulator dot of the CPU oracle.

Zero products leave a pair unchanged (TwoSum(s, 0) = (s, 0) exactly), so
the zeros around the three products do not disturb the cases."""
import numpy as np
import pytest
import torch

import oracle
from dot2_tree import element, plan
from gpu_util import host

pytestmark = pytest.mark.gpu

BIG = (2.0 ** 20, 2.0 ** 20)     # product +2^40
ONE = (1.0, 1.0)                 # product 1
NEG = (-2.0 ** 20, 2.0 ** 20)    # product -2^40


def large_cases(p, aligned=True):
    """Cases of the two-stage form's first stage (workgroup level)."""
    def E(**kw):
        return element(p, aligned=aligned, **kw)
    cases = {"lane chain": ([(E(k=0), BIG), (E(k=1), ONE), (E(k=2), NEG)], 0.0)}
    if aligned:
        cases["components q0,q1"] = ([(E(q=0), BIG), (E(q=1), ONE), (E(q=2), NEG)], 0.0)
        cases["components q2"] = ([(E(q=0), BIG), (E(q=2), ONE), (E(q=3), NEG)], 0.0)
        cases["components q3"] = ([(E(q=0), BIG), (E(q=3), ONE), (E(lane=1), NEG)], 0.0)
    for o in (32, 16, 8, 4, 2, 1):
        later = E(lane=o // 2) if o > 1 else E(w=1)
        cases[f"butterfly xor {o}"] = ([(E(lane=0), BIG), (E(lane=o), ONE), (later, NEG)], 0.0)
    nw = p["NT"] // 64
    for k in range(1, nw):
        later = [(E(w=k + 1), NEG)] if k + 1 < nw else ([(E(b=1), NEG)] if p["nblocks"] > 1 else [])
        cases[f"waves 0..{k}"] = ([(E(w=0), BIG), (E(w=k), ONE)] + later,
                                  0.0 if later else -2.0 ** 40)
    if p["nblocks"] > 1:
        cases["workgroup pair"] = ([(E(k=0), BIG), (E(k=1), ONE), (E(b=1), NEG)], 0.0)
    cases["alpha last"] = ([(E(k=0), NEG), (E(k=1), ONE)], 2.0 ** 40)
    return cases


def stage2_cases(p):
    """Cases of the second stage: per-thread chain over partials i, i + 256,
    ..., its butterfly and its waves (p has 1024 workgroups)."""
    assert p["nblocks"] == 1024

    def W(b):
        return element(p, b=b)
    cases = {
        "stage 2 chain 0,256": ([(W(0), BIG), (W(256), ONE), (W(512), NEG)], 0.0),
        "stage 2 chain 512": ([(W(0), BIG), (W(512), ONE), (W(768), NEG)], 0.0),
        "stage 2 chain 768": ([(W(0), BIG), (W(768), ONE), (W(1), NEG)], 0.0),
    }
    for o in (32, 16, 8, 4, 2, 1):
        later = W(o // 2) if o > 1 else W(64)
        cases[f"stage 2 butterfly xor {o}"] = ([(W(0), BIG), (W(o), ONE), (later, NEG)], 0.0)
    for k in (1, 2, 3):
        later = [(W(64 * (k + 1)), NEG)] if k < 3 else []
        cases[f"stage 2 waves 0..{k}"] = ([(W(0), BIG), (W(64 * k), ONE)] + later, 0.0 if later else -2.0 ** 40)
    return cases


def run_cases(sb, n, cases, offset=0):
    buf_x = torch.zeros(n + offset, dtype=torch.float32, device="cuda")
    buf_y = torch.zeros(n + offset, dtype=torch.float32, device="cuda")
    xd, yd = buf_x[offset:], buf_y[offset:]
    assert (xd.data_ptr() % 16 == 0) == (offset % 4 == 0)
    failures = []
    for name, (entries, alpha0) in cases.items():
        idx = np.array([e for e, _ in entries], dtype=np.int64)
        assert len(set(idx.tolist())) == len(idx) and idx.min() >= 0 and idx.max() < n, (name, idx)
        xs = np.array([v[0] for _, v in entries], np.float32)
        ys = np.array([v[1] for _, v in entries], np.float32)
        it = torch.from_numpy(idx).cuda()
        xd[it], yd[it] = torch.from_numpy(xs).cuda(), torch.from_numpy(ys).cuda()
        a = torch.tensor([alpha0], dtype=torch.float32, device="cuda")
        sb.sb_dot2_f32(xd, yd, a)
        plain = torch.tensor([alpha0], dtype=torch.float32, device="cuda")
        sb.sb_dot(xd, yd, plain)
        got, got_plain = float(host(a)[0]), float(host(plain)[0])
        xd[it], yd[it] = 0.0, 0.0
        exact = oracle.dot_exact_f32(xs, ys, alpha0)   # the zeros add nothing
        assert exact == 1.0, (name, exact)
        if got != exact:
            failures.append(f"{name}: dot2 {got!r}, exact {exact!r}")
        if got_plain == exact:
            failures.append(f"{name}: the plain binary32 DOT also gave {got_plain!r} (case has no teeth)")
    assert not failures, f"n={n} offset={offset}: " + "; ".join(failures)


@pytest.mark.parametrize("n,offset", [(16384, 0), (16383, 1), (65536, 0), (65539, 0), (65537, 1)])
def test_dot2_levels_first_stage(sb, n, offset):
    """Every merge level of one workgroup (and, for the two-stage form, the
    hand-over of the workgroup's pair and alpha's TwoSum), for the single-
    and the two-stage forms, aligned and unaligned operands."""
    p = plan(n)
    aligned = offset == 0
    cases = large_cases(p, aligned)
    if aligned and n % 4:
        # the scalar tail after the last full vector joins thread 0's pair
        b = p["nblocks"] - 1
        b0 = b * p["chunk"]
        tail = b0 + (n - b0) // 4 * 4
        cases["vector tail"] = ([(element(p, b=b), BIG), (tail, ONE), (element(p, b=b, lane=1), NEG)], 0.0)
    run_cases(sb, n, cases, offset)


def test_dot2_levels_second_stage(sb):
    """The second stage's per-thread chain, butterfly and waves, with the
    largest grid (1024 workgroups)."""
    n = 1 << 24
    p = plan(n)
    run_cases(sb, n, stage2_cases(p))
