"""Shared helpers of the GPU parity tests: moving numpy inputs to the
device and the error bounds the results are held to."""
import numpy as np
import torch

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def gamma(k, u):
    return k * u / (1.0 - k * u)


def dev(a, device="cuda"):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def unit(dtype):
    return U64 if dtype in (np.float64, torch.float64) else U32


def gemv_bound(A, x, c0, op, K, u):
    """Per-entry acceptance 2*gamma_{K+1}(u)*(|c0| + sum|a||x|), evaluated in
    binary64: both the GPU result and the oracle lie within
    gamma_{K+1}(|c0| + sum|a||x|) of the exact value for any summation order,
    with or without fused multiply-add."""
    Aa = np.abs(np.asarray(A, dtype=np.float64))
    xa = np.abs(np.asarray(x, dtype=np.float64))
    s = Aa @ xa if op == 0 else Aa.T @ xa
    return 2.0 * gamma(K + 1, u) * (np.abs(np.asarray(c0, dtype=np.float64)) + s)


def assert_within(got, ref, bound, what=""):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    bad = ~(err <= bound)  # NaN counts as bad
    both_nan = np.isnan(got) & np.isnan(ref)
    bad &= ~both_nan
    if bad.any():
        i = int(np.flatnonzero(bad)[0])
        raise AssertionError(f"{what}: {int(bad.sum())} entries out of bound; first at {i}: "
                             f"got {got.flat[i]!r} ref {ref.flat[i]!r} bound {bound.flat[i]!r}")


def normwise(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(got, dtype=np.float64) - ref) / max(np.linalg.norm(ref), 1e-300))
