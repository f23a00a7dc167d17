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


def bucket_errors(got, ref):
    """Largest elementwise relative error by the entry's size relative to the
    largest entry of its column: (>= 1e-3, >= 1e-9, >= 1e-30, smaller)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.ndim == 1:
        ref, got = ref[:, None], got[:, None]
    cmax = np.max(np.abs(ref), axis=0, keepdims=True)
    rel = np.abs(got - ref) / np.where(ref != 0, np.abs(ref), 1.0)
    w = np.abs(ref) / np.where(cmax > 0, cmax, 1.0)
    out = []
    for lo, hi in ((1e-3, np.inf), (1e-9, 1e-3), (1e-30, 1e-9), (0.0, 1e-30)):
        m = (w >= lo) & (w < hi) & (ref != 0) & (np.abs(ref) >= 1e-300)
        out.append(float(rel[m].max()) if m.any() else 0.0)
    return out


def colmax_errors(got, ref):
    """Per column max_i |G - O| / max_i |O| (the largest of them)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.ndim == 1:
        ref, got = ref[:, None], got[:, None]
    cmax = np.max(np.abs(ref), axis=0)
    err = np.max(np.abs(got - ref), axis=0)
    ok = cmax > 0
    return float(np.max(err[ok] / cmax[ok])) if ok.any() else float(np.max(err))


def assert_iterate_parity(got, ref, tol, what=""):
    """Gate for FP64 factor matrices after whole solves (several sweeps over
    all modes): normwise <= tol, column-wise max-norm max_i |G - O| /
    max_i |O| <= tol in every column, and exact zeros kept. An entry the
    iteration drives toward zero belongs to a dying part of the model whose
    factors are products of small numbers across the modes; its relative
    rounding difference grows with each sweep (measured up to 4e-11 on
    entries 1e-70 below their column's largest after six sweeps), while its
    share of the column is negligible, so every entry is held to the scale of
    its column."""
    nw, el, zok = rel_errors(got, ref)
    cm = colmax_errors(got, ref)
    ok = nw <= tol and cm <= tol and zok
    assert ok, (f"{what}: normwise {nw:.3e}, column-wise {cm:.3e}, elementwise {el:.3e} "
                f"(by size {['%.1e' % x for x in bucket_errors(got, ref)]}), zeros ok {zok}")
    return nw, cm, el
