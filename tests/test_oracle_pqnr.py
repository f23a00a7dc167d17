"""Pins of the oracle's PQNR row solves (projected quasi-Newton per row of a
mode; the paper names the variant in its Background, readings in the oracle).

Each row subproblem, min_{b >= 0} sum(b) - sum_k x_k log(b . pi_k), is convex;
with normalised other factors it has a unique minimiser when the row's pi_k
span the rank. The pins check the oracle against things it does not compute
itself: scipy's bound-constrained L-BFGS-B on the same objective (an
independent solver), the closed form at R = 1, the KKT conditions and the
objective's decrease evaluated here in NumPy, and the mass identity."""
import numpy as np
import pytest

from paper_2307_03276_amd import synth
from tests import dense_ref


def _pis(X, mode, factors, rows):
    """pi_k for the nonzeros of each row, from the factors with NumPy."""
    R = factors[0].shape[1]
    out = {}
    for i in rows:
        ks = np.flatnonzero(X.idx[mode] == i)
        p = np.ones((ks.size, R))
        for m in range(X.nmodes):
            if m != mode:
                p *= factors[m][X.idx[m][ks]]
        out[i] = (X.vals[ks], p)
    return out


def _f(b, xs, p, eps=1e-10):
    return float(b.sum() - np.sum(xs * np.log(np.maximum(p @ b, eps))))


def _grad(b, xs, p, eps=1e-10):
    return 1.0 - (xs / np.maximum(p @ b, eps)) @ p


def test_pqnr_matches_independent_lbfgsb(oracle_lib):
    from scipy.optimize import minimize
    X, M, _ = synth.config_small()
    n = 1
    B0 = M.factors[n] * M.lam
    Bq, st = oracle_lib.pqnr_inner(X, n, B0, M.factors, lmax=200, tau=1e-12)
    assert st["last_viol"] < 1e-12
    rows = [0, 7, 33, 61, 79]
    for i, (xs, p) in _pis(X, n, M.factors, rows).items():
        res = minimize(lambda b: _f(b, xs, p), B0[i], jac=lambda b: _grad(b, xs, p), method="L-BFGS-B",
                       bounds=[(0, None)] * p.shape[1], options=dict(ftol=1e-15, gtol=1e-12, maxiter=20000))
        fq, fs = _f(Bq[i], xs, p), _f(res.x, xs, p)
        assert fq <= fs + 1e-9 * abs(fs), (i, fq, fs)
        scale = max(1.0, np.abs(res.x).max())
        assert np.max(np.abs(Bq[i] - res.x)) <= 1e-4 * scale, (i, np.max(np.abs(Bq[i] - res.x)))


def test_pqnr_kkt_at_convergence(oracle_lib):
    X, M, _ = synth.config_small()
    for n in range(3):
        B0 = M.factors[n] * M.lam
        Bq, st = oracle_lib.pqnr_inner(X, n, B0, M.factors, lmax=300, tau=1e-10)
        assert np.all(Bq >= 0)
        G = 1.0 - dense_ref.phi_dense(X, n, Bq, M.factors, 1e-10)  # independent gradient
        assert np.max(np.abs(np.minimum(Bq, G))) < 1e-10
        assert np.all(G > -1e-10)


def test_pqnr_rank_one_closed_form(oracle_lib):
    """R = 1: the row optimum is the row's total count (normalised factors)."""
    X = synth.random_tensor(5, (7, 6, 5), 120)
    M = synth.random_model(5, X.dims, 1)
    for n in range(3):
        Bq, st = oracle_lib.pqnr_inner(X, n, M.factors[n] * M.lam, M.factors, lmax=20, tau=1e-12)
        marg = np.bincount(X.idx[n], weights=X.vals, minlength=X.dims[n])
        np.testing.assert_allclose(Bq[:, 0], marg, rtol=1e-13, atol=0)


def test_pqnr_objective_decreases_every_step(oracle_lib):
    X, M, _ = synth.config_small()
    n = 2
    B0 = M.factors[n] * M.lam
    rows = [3, 17, 42]
    pis = _pis(X, n, M.factors, rows)
    prev = {i: _f(B0[i], *pis[i]) for i in rows}
    for lmax in range(1, 16):
        Bq, _ = oracle_lib.pqnr_inner(X, n, B0, M.factors, lmax=lmax, tau=0.0, rows=rows)
        for i in rows:
            f = _f(Bq[i], *pis[i])
            assert f <= prev[i] + 1e-12 * abs(prev[i]), (lmax, i, f, prev[i])
            prev[i] = f


def test_pqnr_converges_faster_than_mu(oracle_lib):
    """Quasi-Newton: every row of every mode at KKT 1e-8 within 60 steps (MU's
    loop is still above 1e-3 after 2000 iterations on the same rows)."""
    X, M, _ = synth.config_small()
    for n in range(3):
        _, st = oracle_lib.pqnr_inner(X, n, M.factors[n] * M.lam, M.factors, lmax=60, tau=1e-8)
        assert st["last_viol"] < 1e-8 and st["n_updates"] < 60


def test_pqnr_rows_are_independent(oracle_lib):
    X, M, _ = synth.config_small()
    n = 0
    B0 = M.factors[n] * M.lam
    full, _ = oracle_lib.pqnr_inner(X, n, B0, M.factors, lmax=25, tau=1e-6)
    rows = [1, 50, 99]
    part, _ = oracle_lib.pqnr_inner(X, n, B0, M.factors, lmax=25, tau=1e-6, rows=rows)
    np.testing.assert_array_equal(part[rows], full[rows])
    others = np.setdiff1d(np.arange(X.dims[n]), rows)
    np.testing.assert_array_equal(part[others], B0[others])


def test_pqnr_solve_mass_normalisation_and_fit(oracle_lib):
    """A converged PQNR solve: unit column sums, sum(lambda) = sum(x) (the row
    optima satisfy b . g = 0, i.e. sum(b) = sum(b . phi) = the row's counts),
    and a log-likelihood at least that of the MU solve with the same sweeps."""
    X, M, _ = synth.config_small()
    out, st = oracle_lib.pqnr_solve(X, M, kmax=8, lmax=50, tau=1e-9)
    for a in out.factors:
        np.testing.assert_allclose(a.sum(axis=0), 1.0, rtol=1e-12)
    assert abs(out.lam.sum() - X.vals.sum()) <= 1e-7 * X.vals.sum()
    mu, _ = oracle_lib.solve(X, M, kmax=8, lmax=10, tau=0.0)
    assert oracle_lib.loglik(X, out) >= oracle_lib.loglik(X, mu)


# Two one-row subproblems found by a seeded search (a 1 x J x K tensor with
# Zipf(1.1) coordinates): (seed, J, K, nonzeros, R, the first trial whose
# sufficient-decrease test passes at the third step, 0-based). Along that step's
# quasi-Newton direction the first passes at alpha = 1/8 (the fourth and last
# trial of the reading) and at alpha = 1/16 (a fifth trial the reading does not
# make).
CRAFTED = [(100, 13, 10, 50, 2, 3), (571, 15, 9, 42, 3, 4)]


@pytest.mark.parametrize("seed,J,K,nnz,R,first_pass", CRAFTED)
def test_pqnr_line_search_four_trials_then_mu_step(oracle_lib, seed, J, K, nnz, R, first_pass):
    """The trial count and the fallback of the PQNR reading: four backtracking
    trials (alpha = 1 .. 1/8), then the MU step b * phi with the curvature
    pairs dropped. The third step of each crafted row is a quasi-Newton step
    (two pairs, a descent direction): where the fourth trial passes, the
    oracle takes it; where only a fifth would pass, the oracle takes the MU
    step, and the steps after it differ from those keeping the pairs gives."""
    from tests import rowsolve_ref as ref
    X = synth.random_tensor(seed, (1, J, K), nnz, zipf=(None, 1.1, 1.1))
    M = synth.random_model(seed, X.dims, R)
    xs = X.vals
    P = M.factors[1][X.idx[1]] * M.factors[2][X.idx[2]]
    B0 = M.factors[0] * M.lam
    b0 = B0[0]
    orc = [b0] + [oracle_lib.pqnr_inner(X, 0, B0, M.factors, lmax=k, tau=0.0)[0][0] for k in range(1, 7)]
    log = []
    its = ref.pqnr_row(xs, P, b0, 6, log=log)
    for k in range(7):  # the oracle takes the reading's steps
        assert np.max(np.abs(orc[k] - its[k])) <= 1e-13 * np.max(np.abs(its[k])), k
    e = log[2]
    b, g, d = e["b"], e["g"], e["d"]
    assert e["npairs"] == 2 and np.dot(g, d) < 0.0 and not np.allclose(d, -b * g)
    passes = []
    for alpha in (1.0, 0.5, 0.25, 0.125, 0.0625):
        delta = np.maximum(b + alpha * d, 0.0) - b
        gd = float(np.dot(g, delta))
        assert gd < 0.0
        passes.append(ref.objective_change(b, delta, xs, P) <= 1e-4 * gd)
    assert passes.index(True) == first_pass, passes
    phi = (xs / (P @ b)) @ P  # the MU step, from Phi's definition
    if first_pass < 4:
        taken = b + (np.maximum(b + 0.5 ** first_pass * d, 0.0) - b)
        np.testing.assert_allclose(orc[3], taken, rtol=1e-13, atol=0)
        assert np.max(np.abs(orc[3] - b * phi)) > 1e-3 * np.max(np.abs(b * phi))
    else:
        np.testing.assert_allclose(orc[3], b * phi, rtol=1e-13, atol=0)
        fifth = b + (np.maximum(b + 0.0625 * d, 0.0) - b)
        assert np.max(np.abs(orc[3] - fifth)) > 1e-3 * np.max(np.abs(fifth))
        kept = ref.pqnr_row(xs, P, b0, 6, keep_pairs_on_fail=True)
        assert max(np.max(np.abs(orc[k] - kept[k])) / np.max(np.abs(kept[k])) for k in range(4, 7)) > 1e-6
