"""Pins of the oracle's PDNR row solves (projected damped Newton per row of a
mode with the row's exact Hessian; the paper names the variant in its
Background, readings in the oracle's PDNR section).

The row subproblem is the one PQNR solves, min_{b >= 0} sum(b) - sum_k x_k
log(b . pi_k). Pins: an independent bound-constrained solver (scipy's
L-BFGS-B), the closed form at R = 1, KKT and objective decrease evaluated here
in NumPy, the first step against a damped Newton step built here from a
finite-difference Hessian and NumPy's dense solver, Newton's fast local
convergence, and the mass identity of a converged solve."""
import numpy as np
import pytest

from paper_2307_03276_amd import synth
from tests import dense_ref
from tests.test_oracle_pqnr import _f, _grad, _pis

# Readings fixed by the oracle's PDNR section: initial damping, held-entry
# threshold, sufficient-decrease constant, trials.
MU0, HELD, SIGMA, TRIALS = 1e-3, 1e-10, 1e-4, 4


def test_pdnr_matches_independent_lbfgsb(oracle_lib):
    from scipy.optimize import minimize
    X, M, _ = synth.config_small()
    n = 1
    B0 = M.factors[n] * M.lam
    Bd, st = oracle_lib.pdnr_inner(X, n, B0, M.factors, lmax=200, tau=1e-12)
    assert st["last_viol"] < 1e-12
    rows = [0, 7, 33, 61, 79]
    for i, (xs, p) in _pis(X, n, M.factors, rows).items():
        res = minimize(lambda b: _f(b, xs, p), B0[i], jac=lambda b: _grad(b, xs, p), method="L-BFGS-B",
                       bounds=[(0, None)] * p.shape[1], options=dict(ftol=1e-15, gtol=1e-12, maxiter=20000))
        fd, fs = _f(Bd[i], xs, p), _f(res.x, xs, p)
        assert fd <= fs + 1e-9 * abs(fs), (i, fd, fs)
        scale = max(1.0, np.abs(res.x).max())
        assert np.max(np.abs(Bd[i] - res.x)) <= 1e-4 * scale, (i, np.max(np.abs(Bd[i] - res.x)))


def test_pdnr_kkt_at_convergence(oracle_lib):
    X, M, _ = synth.config_small()
    for n in range(3):
        B0 = M.factors[n] * M.lam
        Bd, st = oracle_lib.pdnr_inner(X, n, B0, M.factors, lmax=300, tau=1e-10)
        assert np.all(Bd >= 0)
        G = 1.0 - dense_ref.phi_dense(X, n, Bd, M.factors, 1e-10)  # independent gradient
        assert np.max(np.abs(np.minimum(Bd, G))) < 1e-10
        assert np.all(G > -1e-10)
        np.testing.assert_allclose(st["phi_last"], 1.0 - G, rtol=0, atol=1e-9)


@pytest.mark.parametrize("dims,R,nnz", [((12, 10, 8, 6), 5, 1500), ((7, 6, 5, 4, 3), 3, 600)])
def test_pdnr_kkt_at_convergence_more_modes(oracle_lib, dims, R, nnz):
    """Four and five modes (pi from three and four other factors)."""
    X = synth.random_tensor(21, dims, nnz)
    M = synth.random_model(21, dims, R)
    for n in range(len(dims)):
        B0 = M.factors[n] * M.lam
        Bd, st = oracle_lib.pdnr_inner(X, n, B0, M.factors, lmax=200, tau=1e-10)
        assert np.all(Bd >= 0)
        G = 1.0 - dense_ref.phi_dense(X, n, Bd, M.factors, 1e-10)
        assert np.max(np.abs(np.minimum(Bd, G))) < 1e-10, n
        assert np.all(G > -1e-10)


def test_pdnr_rank_one_closed_form(oracle_lib):
    """R = 1: the row optimum is the row's total count (normalised factors)."""
    X = synth.random_tensor(5, (7, 6, 5), 120)
    M = synth.random_model(5, X.dims, 1)
    for n in range(3):
        Bd, st = oracle_lib.pdnr_inner(X, n, M.factors[n] * M.lam, M.factors, lmax=30, tau=0.0)
        marg = np.bincount(X.idx[n], weights=X.vals, minlength=X.dims[n])
        np.testing.assert_allclose(Bd[:, 0], marg, rtol=1e-13, atol=0)


def test_pdnr_objective_decreases_every_step(oracle_lib):
    X, M, _ = synth.config_small()
    n = 2
    B0 = M.factors[n] * M.lam
    rows = [3, 17, 42]
    pis = _pis(X, n, M.factors, rows)
    prev = {i: _f(B0[i], *pis[i]) for i in rows}
    for lmax in range(1, 12):
        Bd, _ = oracle_lib.pdnr_inner(X, n, B0, M.factors, lmax=lmax, tau=0.0, rows=rows)
        for i in rows:
            f = _f(Bd[i], *pis[i])
            assert f <= prev[i] + 1e-12 * abs(prev[i]), (lmax, i, f, prev[i])
            prev[i] = f


def _fd_hessian(b, xs, p, h_rel=1e-6):
    """Central differences of the NumPy gradient: an independent Hessian."""
    R = b.size
    H = np.empty((R, R))
    for r in range(R):
        h = h_rel * max(abs(b[r]), 1.0)
        e = np.zeros(R)
        e[r] = h
        H[:, r] = (_grad(b + e, xs, p) - _grad(b - e, xs, p)) / (2 * h)
    return 0.5 * (H + H.T)


def _first_step(b, xs, p, H):
    """One PDNR iteration from b built here: held set, damped Newton system on
    the free set solved by NumPy, projected backtracking."""
    g = _grad(b, xs, p)
    held = (g > 0) & (b <= HELD)
    F = np.flatnonzero(~held)
    d = -g.copy()
    t = np.trace(H[np.ix_(F, F)]) / F.size
    K = H[np.ix_(F, F)] + MU0 * t * np.eye(F.size)
    d[F] = np.linalg.solve(K, -g[F])
    assert g @ d < 0
    f0 = _f(b, xs, p)
    for k in range(TRIALS):
        delta = np.maximum(b + 0.5 ** k * d, 0.0) - b
        gd = g @ delta
        if gd < 0 and np.all(p @ (b + delta) > 1e-10) and _f(b + delta, xs, p) - f0 <= SIGMA * gd:
            return b + delta
    return None


def test_pdnr_first_step_is_damped_newton(oracle_lib):
    """From the same start, the oracle's first step equals a damped projected
    Newton step built here: with the exact Hessian (NumPy outer products) to
    1e-10, and with a finite-difference Hessian of the NumPy gradient to 1e-5
    (which pins the Hessian's formula independently of its algebra)."""
    X, M, _ = synth.config_small()
    n = 0
    B0 = M.factors[n] * M.lam
    rows = [2, 11, 40, 77, 95]
    Bd, _ = oracle_lib.pdnr_inner(X, n, B0, M.factors, lmax=1, tau=0.0, rows=rows)
    checked = 0
    for i, (xs, p) in _pis(X, n, M.factors, rows).items():
        if xs.size < p.shape[1]:
            continue
        m = p @ B0[i]
        H = (p * (xs / m ** 2)[:, None]).T @ p
        want = _first_step(B0[i], xs, p, H)
        if want is None:
            continue
        scale = np.abs(want).max()
        assert np.max(np.abs(Bd[i] - want)) <= 1e-10 * scale, (i, np.max(np.abs(Bd[i] - want)) / scale)
        want_fd = _first_step(B0[i], xs, p, _fd_hessian(B0[i], xs, p))
        assert np.max(np.abs(Bd[i] - want_fd)) <= 1e-5 * scale, (i, np.max(np.abs(Bd[i] - want_fd)) / scale)
        checked += 1
    assert checked >= 3


def test_pdnr_converges_in_few_steps(oracle_lib):
    """Newton: every row of every mode at KKT 1e-10 within 40 steps, and
    fewer steps over all rows than PQNR needs for the same tolerance."""
    X, M, _ = synth.config_small()
    for n in range(3):
        B0 = M.factors[n] * M.lam
        _, st = oracle_lib.pdnr_inner(X, n, B0, M.factors, lmax=40, tau=1e-10)
        assert st["last_viol"] < 1e-10 and st["n_updates"] < 40, (n, st["last_viol"], st["n_updates"])
        _, sq = oracle_lib.pqnr_inner(X, n, B0, M.factors, lmax=200, tau=1e-10)
        assert st["row_steps"] < sq["row_steps"], (n, st["row_steps"], sq["row_steps"])


def test_pdnr_empty_rows_go_to_zero(oracle_lib):
    """A row without nonzeros has f = sum(b): one MU step takes it to 0."""
    X = synth.random_tensor(3, (9, 6, 5), 40)
    keep = X.idx[0] != 4
    X = synth.SparseTensor(X.dims, np.ascontiguousarray(X.idx[:, keep]), X.vals[keep].copy())
    M = synth.random_model(3, X.dims, 4)
    Bd, st = oracle_lib.pdnr_inner(X, 0, M.factors[0] * M.lam, M.factors, lmax=1, tau=0.0)
    assert np.all(Bd[4] == 0.0)


def test_pdnr_rows_are_independent(oracle_lib):
    X, M, _ = synth.config_small()
    n = 0
    B0 = M.factors[n] * M.lam
    full, _ = oracle_lib.pdnr_inner(X, n, B0, M.factors, lmax=25, tau=1e-6)
    rows = [1, 50, 99]
    part, _ = oracle_lib.pdnr_inner(X, n, B0, M.factors, lmax=25, tau=1e-6, rows=rows)
    np.testing.assert_array_equal(part[rows], full[rows])
    others = np.setdiff1d(np.arange(X.dims[n]), rows)
    np.testing.assert_array_equal(part[others], B0[others])


def test_pdnr_solve_mass_normalisation_and_fit(oracle_lib):
    """A converged PDNR solve: unit column sums, sum(lambda) = sum(x), and a
    log-likelihood at least that of the MU solve with the same sweeps."""
    X, M, _ = synth.config_small()
    out, st = oracle_lib.pdnr_solve(X, M, kmax=8, lmax=30, tau=1e-9)
    for a in out.factors:
        np.testing.assert_allclose(a.sum(axis=0), 1.0, rtol=1e-12)
    assert abs(out.lam.sum() - X.vals.sum()) <= 1e-7 * X.vals.sum()
    mu, _ = oracle_lib.solve(X, M, kmax=8, lmax=10, tau=0.0)
    assert oracle_lib.loglik(X, out) >= oracle_lib.loglik(X, mu)
