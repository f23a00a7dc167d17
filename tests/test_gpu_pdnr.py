"""PDNR row solves on the GPU against the oracle's PDNR (same row rules).

Every decision of a row (KKT stop, held set, Cholesky pivots, descent test,
sufficient decrease, damping update) is taken from quantities both sides form
to within rounding, so short schedules run in lockstep: step counts match and
the iterates agree normwise to the parity tolerance. The damped Newton
systems have condition numbers up to about R / mu, so the lockstep gate is
that amplification of one rounding (1e-12 at the least), and long runs are
compared where both sides converge: within tol of KKT at the same row
optimum."""
import numpy as np
import pytest

import oracle
from paper_2307_03276_amd import cpapr, synth
from tests.gpu_util import assert_parity, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available()
    oracle.build(force=False)
    cpapr.load()


def _plan(X, R, **kw):
    return cpapr.Plan.from_tensor(X, R, method=cpapr.CPAPR_METHOD_PDNR, **kw)


U = 2.0 ** -53  # FP64 unit roundoff
MU0, MU_STEP = 1e-3, 4.0  # the damping's start and factor (cpapr.h, CPAPR_METHOD_PDNR)


def _lockstep_tol(R, lmax):
    """Rounding of the damped Newton solve is amplified by the system's
    condition number, at most 1 + R / mu for H_FF + mu t I with t the mean
    diagonal; after l - 1 accepted steps mu >= MU0 / MU_STEP^(l-1). The parity
    gate is that amplification of one unit roundoff, and never below 1e-12."""
    return max(1e-12, U * (1.0 + R * MU_STEP ** (lmax - 1) / MU0))


def _lockstep(X, M, R, lmax):
    tol_rel = _lockstep_tol(R, lmax)
    P = _plan(X, R, lmax=lmax, tol=0.0)  # fixed schedule: every row steps lmax times
    A = [dev(a) for a in M.factors]
    for n in range(X.nmodes):
        Bh = M.factors[n] * M.lam
        B = dev(Bh)
        st = P.pdnr_inner(n, B, A)
        Bo, ost = oracle.pdnr_inner(X, n, Bh, M.factors, lmax=lmax, tau=0.0)
        assert st["inner_iters"] == ost["n_updates"] == lmax
        assert st["row_steps"] == ost["row_steps"]
        assert st["phi_evals"] == lmax
        # normwise: a projected step can leave an entry at a tiny value formed by
        # cancellation (b + (max(b + alpha d, 0) - b)), whose relative error says nothing
        got = host(B)
        err = np.max(np.abs(got - Bo)) / np.max(np.abs(Bo))
        assert err <= tol_rel, f"B after {lmax} PDNR steps, mode {n}: {err:.2e}"
    P.close()


@pytest.mark.parametrize("lmax", [1, 2, 4])
def test_pdnr_short_schedule_lockstep(lmax):
    X, M, _ = synth.config_small()
    _lockstep(X, M, 10, lmax)


@pytest.mark.parametrize("dims,R,nnz", [((6, 5, 4, 3, 5, 4, 3, 2), 3, 500), ((40, 30, 20, 10), 4, 3000),
                                        ((30, 20, 10), 64, 4000), ((50, 40, 30), 33, 6000),
                                        ((120, 90), 8, 3000)])
def test_pdnr_unusual_shapes_lockstep(dims, R, nnz):
    """Eight modes; the largest rank (a full 64-lane system); a rank one past a
    power of two (padded system); a matrix (pi from one other factor)."""
    X = synth.random_tensor(41, dims, nnz)
    M = synth.random_model(41, dims, R)
    _lockstep(X, M, R, 2)


def test_pdnr_heavy_rows_cross_tiles_lockstep():
    """Zipf rows of thousands of nonzeros span several tiles of the Hessian
    pass, whose ends meet by atomics."""
    X = synth.random_tensor(13, (300, 200, 100), 60_000, zipf=(1.4, None, None))
    M = synth.random_model(13, X.dims, 16)
    assert np.bincount(X.idx[0]).max() > 2048
    _lockstep(X, M, 16, 2)


@pytest.mark.parametrize("dims,R,nnz", [((100, 80, 60), 10, 10_000), ((40, 30, 20, 10), 4, 3000),
                                        ((60, 50, 40), 32, 8000), ((200, 100, 80), 16, 40_000)])
def test_pdnr_converged_rows_match_oracle(dims, R, nnz):
    X = synth.random_tensor(11, dims, nnz, zipf=(1.1,) + (None,) * (len(dims) - 1))
    M = synth.random_model(11, dims, R)
    tau = 1e-9
    P = _plan(X, R, lmax=100, tol=tau)
    A = [dev(a) for a in M.factors]
    for n in range(len(dims)):
        Bh = M.factors[n] * M.lam
        B = dev(Bh)
        st = P.pdnr_inner(n, B, A)
        Bo, ost = oracle.pdnr_inner(X, n, Bh, M.factors, lmax=100, tau=tau)
        assert st["kkt_violation"] < tau and ost["last_viol"] < tau
        assert st["converged"] == 1
        # a row whose violation lands within rounding of tau may stop one step
        # earlier or later on either side
        assert abs(st["row_steps"] - ost["row_steps"]) <= max(4, ost["row_steps"] // 50)
        assert_parity(host(B), Bo, 1e-6, f"converged B mode {n}", elementwise=False)
    P.close()


def test_pdnr_rank_one_and_empty_rows():
    """R = 1: the iterates reach the row totals; rows without nonzeros go to
    zero at the first step."""
    X = synth.random_tensor(5, (50, 40, 30), 300)
    M = synth.random_model(5, X.dims, 1)
    P = _plan(X, 1, lmax=30, tol=0.0)
    A = [dev(a) for a in M.factors]
    for n in range(3):
        B = dev(M.factors[n] * M.lam)
        P.pdnr_inner(n, B, A)
        marg = np.bincount(X.idx[n], weights=X.vals, minlength=X.dims[n])
        got = host(B)[:, 0]
        np.testing.assert_allclose(got, marg, rtol=1e-12, atol=0)
        assert np.all(got[marg == 0] == 0.0)
    P.close()


def test_pdnr_solve_matches_oracle():
    X, M, _ = synth.config_small()
    P = _plan(X, 10, kmax=3, lmax=3, tol=0.0)
    lam = dev(M.lam)
    A = [dev(a) for a in M.factors]
    st = P.solve(lam, A)
    out, ost = oracle.pdnr_solve(X, M, kmax=3, lmax=3, tau=0.0)
    assert st["outer_iters"] == ost["outer_iters"] == 3
    assert st["row_steps"] == ost["row_steps"]
    assert_parity(host(lam), out.lam, 1e-10, "lambda")
    for n in range(3):
        assert_parity(host(A[n]), out.factors[n], 1e-10, f"A{n}", elementwise=False)
    assert st["phi_evals"] == 3 * 3 * 3
    P.close()


def test_pdnr_solve_reaches_lower_kkt_than_pqnr_and_mu():
    """Same outer sweeps and inner limit: the PDNR solve ends closer to a KKT
    point than PQNR and MU, above MU's likelihood, and at the oracle's
    likelihood. (The outer problem is not convex: PDNR and PQNR can settle at
    slightly different points, so their likelihoods are not ordered.)"""
    X, M, _ = synth.config_small()
    kw = dict(kmax=10, lmax=10, tol=1e-6)
    out = {}
    for name, method in (("pdnr", cpapr.CPAPR_METHOD_PDNR), ("pqnr", cpapr.CPAPR_METHOD_PQNR),
                         ("mu", cpapr.CPAPR_METHOD_MU)):
        P = cpapr.Plan.from_tensor(X, 10, method=method, **kw)
        lam, A = dev(M.lam), [dev(a) for a in M.factors]
        out[name] = P.solve(lam, A)
        P.close()
    assert out["pdnr"]["kkt_violation"] < out["pqnr"]["kkt_violation"] < out["mu"]["kkt_violation"]
    assert out["pdnr"]["loglik"] >= out["mu"]["loglik"]
    o, _ = oracle.pdnr_solve(X, M, kmax=10, lmax=10, tau=1e-6)
    assert abs(out["pdnr"]["loglik"] - oracle.loglik(X, o)) <= 1e-6 * abs(out["pdnr"]["loglik"])


def test_pdnr_rejects_other_plans_and_settings():
    X, M, _ = synth.config_small()
    P = cpapr.Plan.from_tensor(X, 10, method=cpapr.CPAPR_METHOD_PQNR)
    with pytest.raises(cpapr.CpaprError) as ei:
        P.pdnr_inner(0, dev(M.factors[0] * M.lam), [dev(a) for a in M.factors])
    assert ei.value.code == -1
    P.close()
    for kw in (dict(precision=cpapr.CPAPR_MIXED), dict(deterministic=1)):
        with pytest.raises(cpapr.CpaprError) as ei:
            _plan(X, 10, **kw)
        assert ei.value.code == -6
    X2 = synth.random_tensor(3, (20, 10, 10), 500)
    with pytest.raises(cpapr.CpaprError) as ei:
        _plan(X2, 65)
    assert ei.value.code == -6
