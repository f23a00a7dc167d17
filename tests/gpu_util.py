"""Helpers shared by the GPU parity tests: moving seeded inputs to the device and
comparing against the oracle under the parity gate."""
import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel_errors(got, ref, floor=1e-100):
    """(normwise ||G-O||_F/||O||_F, elementwise max |G-O|/|O| over |O| >= floor,
    and whether G is exactly 0 wherever O is exactly 0)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape
    assert np.all(np.isfinite(got)), "non-finite values in the GPU result"
    nref = np.linalg.norm(ref)
    normwise = np.linalg.norm(got - ref) / nref if nref > 0 else np.linalg.norm(got)
    mask = np.abs(ref) >= floor
    elem = float(np.max(np.abs(got[mask] - ref[mask]) / np.abs(ref[mask]))) if mask.any() else 0.0
    zeros_ok = bool(np.all(got[ref == 0] == 0))
    return float(normwise), elem, zeros_ok


def assert_parity(got, ref, tol, what="", elementwise=True):
    """Gate: normwise relative error <= tol, exact zeros kept, and (unless
    elementwise=False, used for factor matrices of mixed-precision solves,
    whose tiny decaying entries carry FP32 storage error) the elementwise
    relative error <= tol as well."""
    nw, el, zok = rel_errors(got, ref)
    ok = nw <= tol and zok and (el <= tol or not elementwise)
    assert ok, f"{what}: normwise {nw:.3e}, elementwise {el:.3e}, zeros ok {zok}"
    return nw, el
