"""FP64 CPU oracle for CP-APR MU (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
use this package. It wraps the plain single-threaded C in ``cpapr_oracle.c``
(built with gcc by :func:`build`) and takes NumPy arrays; it shares no code
with the GPU library.

Every function follows the paper's definitions (arXiv:2307.03276):
``phi`` is Algorithm 2 evaluated per nonzero; ``mu_inner`` and ``solve`` are the
inner and outer loops of Algorithm 1; ``loglik`` is the Poisson
log-likelihood used for evaluation; ``mttkrp`` is Eqs. 10-12.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpapr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: no fast-math, no FMA contraction."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
    return _lib


_dp = C.POINTER(C.c_double)


class _Kruskal:
    """Result model of :func:`solve`: ``lam`` (R,) and ``factors`` [(I_m, R)]."""

    def __init__(self, lam, factors):
        self.lam = lam
        self.factors = factors

    @property
    def rank(self):
        return int(self.lam.shape[0])


def _ptr(a, ctype=C.c_double):
    return a.ctypes.data_as(C.POINTER(ctype))


def _tensor_args(X):
    idx = np.ascontiguousarray(X.idx, dtype=np.int32)
    vals = np.ascontiguousarray(X.vals, dtype=np.float64)
    dims = np.asarray(X.dims, dtype=np.int64)
    return idx, vals, dims, (C.c_int(len(X.dims)), _ptr(dims, C.c_int64), C.c_int64(vals.shape[0]),
                             _ptr(idx, C.c_int32), _ptr(vals))


def _fac_array(factors):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in factors]
    ptrs = (_dp * len(arrs))(*[_ptr(a) for a in arrs])
    return arrs, ptrs


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with code {rc}")


def phi(X, mode, B, factors, eps=1e-10, rows=None):
    """Phi(n) = (X_(n) ./ max(B Pi, eps)) Pi^T (Algorithm 2). ``rows``: optional
    index array; then only those rows are computed and the rest are NaN."""
    lib = _load()
    keep = _tensor_args(X)
    R = B.shape[1]
    B = np.ascontiguousarray(B, dtype=np.float64)
    arrs, ptrs = _fac_array(factors)
    In = X.dims[mode]
    out = np.full((In, R), np.nan) if rows is not None else np.empty((In, R))
    mask = None
    if rows is not None:
        mask = np.zeros(In, dtype=np.uint8)
        mask[np.asarray(rows)] = 1
    rc = lib.oracle_phi_rows(*keep[3], C.c_int(mode), C.c_int(R), _ptr(B), ptrs, C.c_double(eps),
                             _ptr(mask, C.c_uint8) if mask is not None else None, _ptr(out))
    _check(rc, "phi")
    return out


def mu_inner(X, mode, B, factors, lmax, tau=0.0, eps=1e-10, rows=None):
    """Inner loop of Algorithm 1 for one mode. Returns (B, Phi_last, viol_hist, n_updates).
    With ``rows`` (only valid for tau <= 0) the loop runs on those rows only."""
    if rows is not None and tau > 0:
        raise ValueError("row-restricted inner loop is exact only for tau <= 0")
    lib = _load()
    keep = _tensor_args(X)
    R = B.shape[1]
    Bw = np.array(B, dtype=np.float64, copy=True, order="C")
    arrs, ptrs = _fac_array(factors)
    In = X.dims[mode]
    phi_last = np.zeros((In, R))
    hist = np.full(lmax, np.nan)
    nup = C.c_int(0)
    last = C.c_double(0)
    mask = None
    if rows is not None:
        mask = np.zeros(In, dtype=np.uint8)
        mask[np.asarray(rows)] = 1
    rc = lib.oracle_mu_inner_rows(*keep[3], C.c_int(mode), C.c_int(R), _ptr(Bw), ptrs, C.c_int(lmax),
                                  C.c_double(tau), C.c_double(eps),
                                  _ptr(mask, C.c_uint8) if mask is not None else None,
                                  _ptr(phi_last), _ptr(hist), C.byref(nup), C.byref(last))
    _check(rc, "mu_inner")
    return Bw, phi_last, hist, int(nup.value)


def solve(X, model, kmax, lmax, tau=0.0, eps=1e-10, kappa=0.01, kappa_tol=1e-10):
    """Algorithm 1. Returns (model, stats dict); the input model is not modified."""
    lib = _load()
    keep = _tensor_args(X)
    lam = np.array(model.lam, dtype=np.float64, copy=True)
    arrs, ptrs = _fac_array([a.copy() for a in model.factors])
    outer = C.c_int(0)
    inner = C.c_int64(0)
    conv = C.c_int(0)
    kkt = C.c_double(0)
    rc = lib.oracle_solve(*keep[3], C.c_int(model.rank), _ptr(lam), ptrs, C.c_int(kmax), C.c_int(lmax),
                          C.c_double(tau), C.c_double(eps), C.c_double(kappa), C.c_double(kappa_tol),
                          C.byref(outer), C.byref(inner), C.byref(conv), C.byref(kkt))
    _check(rc, "solve")
    return _Kruskal(lam, arrs), dict(outer_iters=outer.value, inner_updates=inner.value,
                                  converged=bool(conv.value), kkt=kkt.value)


def loglik(X, model, eps=1e-10):
    lib = _load()
    keep = _tensor_args(X)
    lam = np.ascontiguousarray(model.lam, dtype=np.float64)
    arrs, ptrs = _fac_array(model.factors)
    out = C.c_double(0)
    rc = lib.oracle_loglik(*keep[3], C.c_int(model.rank), _ptr(lam), ptrs, C.c_double(eps), C.byref(out))
    _check(rc, "loglik")
    return out.value


def mttkrp(X, mode, factors):
    """M = X_(n) (Khatri-Rao of the other factors) (Eqs. 10-12)."""
    lib = _load()
    keep = _tensor_args(X)
    arrs, ptrs = _fac_array(factors)
    R = arrs[0].shape[1]
    out = np.empty((X.dims[mode], R))
    rc = lib.oracle_mttkrp(*keep[3], C.c_int(mode), C.c_int(R), ptrs, _ptr(out))
    _check(rc, "mttkrp")
    return out


def _rows_inner(fn, X, mode, B, factors, lmax, tau, eps, rows):
    lib = _load()
    keep = _tensor_args(X)
    R = B.shape[1]
    Bw = np.array(B, dtype=np.float64, copy=True, order="C")
    arrs, ptrs = _fac_array(factors)
    In = X.dims[mode]
    mask = None
    if rows is not None:
        mask = np.zeros(In, dtype=np.uint8)
        mask[np.asarray(rows)] = 1
    nup = C.c_int(0)
    total = C.c_int64(0)
    last = C.c_double(0)
    steps = np.zeros(In, dtype=np.int32)
    phi_last = np.full((In, R), np.nan) if rows is not None else np.zeros((In, R))
    rc = getattr(lib, fn)(*keep[3], C.c_int(mode), C.c_int(R), _ptr(Bw), ptrs, C.c_int(lmax),
                          C.c_double(tau), C.c_double(eps),
                          _ptr(mask, C.c_uint8) if mask is not None else None,
                          C.byref(nup), C.byref(total), C.byref(last), _ptr(steps, C.c_int32),
                          _ptr(phi_last))
    _check(rc, fn)
    return Bw, dict(n_updates=int(nup.value), row_steps=int(total.value), last_viol=last.value, steps=steps,
                    phi_last=phi_last)


def _rows_solve(fn, X, model, kmax, lmax, tau, eps, kappa, kappa_tol):
    lib = _load()
    keep = _tensor_args(X)
    lam = np.array(model.lam, dtype=np.float64, copy=True)
    arrs, ptrs = _fac_array([a.copy() for a in model.factors])
    outer = C.c_int(0)
    steps = C.c_int64(0)
    conv = C.c_int(0)
    kkt = C.c_double(0)
    rc = getattr(lib, fn)(*keep[3], C.c_int(model.rank), _ptr(lam), ptrs, C.c_int(kmax), C.c_int(lmax),
                          C.c_double(tau), C.c_double(eps), C.c_double(kappa), C.c_double(kappa_tol),
                          C.byref(outer), C.byref(steps), C.byref(conv), C.byref(kkt))
    _check(rc, fn)
    return _Kruskal(lam, arrs), dict(outer_iters=outer.value, row_steps=steps.value,
                                  converged=bool(conv.value), kkt=kkt.value)


def pqnr_inner(X, mode, B, factors, lmax, tau=0.0, eps=1e-10, rows=None):
    """PQNR row solves of one mode (projected quasi-Newton per row of B; the
    paper names the variant in its Background). Rows are independent, so
    ``rows`` restricts the work exactly for any tau. Returns (B, stats) with
    stats: n_updates (most steps of any row), row_steps (sum over rows),
    last_viol (largest last KKT violation over rows), steps (per row),
    phi_last (the last Phi row computed per row)."""
    return _rows_inner("oracle_pqnr_inner_rows", X, mode, B, factors, lmax, tau, eps, rows)


def pqnr_solve(X, model, kmax, lmax, tau=0.0, eps=1e-10, kappa=0.01, kappa_tol=1e-10):
    """CP-APR with PQNR row solves in place of the MU inner loop (Algorithm 1's
    outer loop, S shift included). Returns (model, stats dict); the input model
    is not modified."""
    return _rows_solve("oracle_pqnr_solve", X, model, kmax, lmax, tau, eps, kappa, kappa_tol)


def pdnr_inner(X, mode, B, factors, lmax, tau=0.0, eps=1e-10, rows=None):
    """PDNR row solves of one mode (projected damped Newton per row of B with
    the row's exact Hessian; the other row-wise variant the Background names).
    Same arguments and results as :func:`pqnr_inner`."""
    return _rows_inner("oracle_pdnr_inner_rows", X, mode, B, factors, lmax, tau, eps, rows)


def pdnr_solve(X, model, kmax, lmax, tau=0.0, eps=1e-10, kappa=0.01, kappa_tol=1e-10):
    """CP-APR with PDNR row solves in place of the MU inner loop (Algorithm 1's
    outer loop, S shift included). Returns (model, stats dict)."""
    return _rows_solve("oracle_pdnr_solve", X, model, kmax, lmax, tau, eps, kappa, kappa_tol)
