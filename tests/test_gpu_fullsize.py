"""Parity at full benchmark size (3-way 200k x 150k x 20k, 20M Zipf(1.1)
nonzeros, R = 16) in the launch configuration the benchmark times.

The oracle computes sampled rows one by one (Phi rows and, because the inner
loop is row-separable under a fixed schedule, inner-loop rows); the mass
identity sum(B .* Phi) = sum(x) checks every row at once."""
import numpy as np
import pytest

import oracle
from paper_2307_03276_amd import cpapr, synth
from tests.gpu_util import assert_parity, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    import torch
    assert torch.cuda.is_available()
    oracle.build(force=False)
    X, M, sched = synth.config_zipf3()
    return X, M, sched


def _sample_rows(X, n, rng, k_random=24):
    counts = np.bincount(X.idx[n], minlength=X.dims[n])
    heavy = np.argsort(counts)[-6:]
    nonempty = np.flatnonzero(counts)
    empty = np.flatnonzero(counts == 0)
    pick = [heavy, rng.choice(nonempty, size=k_random, replace=False)]
    if empty.size:
        pick.append(rng.choice(empty, size=min(4, empty.size), replace=False))
    return np.unique(np.concatenate(pick)), counts


@pytest.mark.parametrize("precision,tol", [(cpapr.CPAPR_FP64, 1e-12), (cpapr.CPAPR_MIXED, 1e-5)])
def test_phi_fullsize_sampled_rows_and_mass(big, precision, tol):
    X, M, sched = big
    P = cpapr.Plan.from_tensor(X, M.rank, precision=precision, lmax=sched["lmax"], tol=0.0)
    A = [dev(a) for a in M.factors]
    rng = np.random.default_rng(0)
    total = X.vals.sum()
    for n in range(3):
        Bh = M.factors[n] * M.lam
        got = host(P.phi(n, dev(Bh), A))
        rows, counts = _sample_rows(X, n, rng)
        ref = oracle.phi(X, n, Bh, M.factors, rows=rows)
        assert_parity(got[rows], ref[rows], tol, f"mode {n} sampled rows")
        mass = float(np.sum(Bh * got))
        assert abs(mass - total) <= tol * total, f"mode {n} mass {mass} vs {total}"
        assert np.all(got[counts == 0] == 0)
    P.close()


def _mttkrp_rows(X, n, rows, factors):
    """The oracle's MTTKRP rows `rows` of mode n, from the nonzeros in them."""
    sel = np.isin(X.idx[n], rows)
    Xs = synth.SparseTensor(X.dims, np.ascontiguousarray(X.idx[:, sel]), X.vals[sel].copy())
    return oracle.mttkrp(Xs, n, factors)[rows]


def test_mttkrp_fullsize_sampled_rows_and_weighted_sum(big):
    """MTTKRP (Eqs. 10-12) at full size in the launch shape the benchmark
    times: sampled rows against the oracle, empty rows exactly zero, and every
    row at once through sum_ir M[i,r] A(n)[i,r] lambda_r = sum_k x_k m_k, the
    model's value summed over the nonzeros weighted by x (computed here from
    the definition, in chunks)."""
    X, M, _ = big
    P = cpapr.Plan.from_tensor(X, M.rank)
    A = [dev(a) for a in M.factors]
    rng = np.random.default_rng(3)
    xm = 0.0
    for c in range(0, X.nnz, 1 << 21):
        m = np.broadcast_to(M.lam, (min(1 << 21, X.nnz - c), M.rank)).copy()
        for q in range(3):
            m *= M.factors[q][X.idx[q, c:c + (1 << 21)]]
        xm += float(X.vals[c:c + (1 << 21)] @ m.sum(axis=1))
    for n in range(3):
        got = host(P.mttkrp(n, A))
        rows, counts = _sample_rows(X, n, rng)
        assert_parity(got[rows], _mttkrp_rows(X, n, rows, M.factors), 1e-12, f"MTTKRP mode {n} sampled rows")
        assert np.all(got[counts == 0] == 0)
        ws = float(np.sum(got * (M.factors[n] * M.lam)))
        assert abs(ws - xm) <= 1e-12 * xm, f"mode {n}: weighted sum {ws} vs {xm}"
    P.close()


def test_mu_inner_fullsize_sampled_rows(big):
    X, M, sched = big
    P = cpapr.Plan.from_tensor(X, M.rank, lmax=sched["lmax"], tol=0.0)
    A = [dev(a) for a in M.factors]
    rng = np.random.default_rng(1)
    n = 0
    Bh = M.factors[n] * M.lam
    B = dev(Bh)
    phi_last, st = P.mu_inner(n, B, A)
    assert st["inner_iters"] == sched["lmax"]
    rows, _ = _sample_rows(X, n, rng, k_random=12)
    Bo, Po, _, _ = oracle.mu_inner(X, n, Bh, M.factors, lmax=sched["lmax"], rows=rows)
    assert_parity(host(B)[rows], Bo[rows], 1e-12, "B rows")
    assert_parity(host(phi_last)[rows], Po[rows], 1e-12, "Phi rows")
    P.close()


def test_pqnr_inner_fullsize_sampled_rows(big):
    """PQNR row solves of mode 0 at full size; rows are independent, so the
    oracle solves the sampled rows alone (heavy rows of 2.6M nonzeros among
    them) with the same tolerance and iteration limit."""
    X, M, sched = big
    P = cpapr.Plan.from_tensor(X, M.rank, method=cpapr.CPAPR_METHOD_PQNR, lmax=8, tol=1e-6)
    A = [dev(a) for a in M.factors]
    rng = np.random.default_rng(2)
    n = 0
    Bh = M.factors[n] * M.lam
    B = dev(Bh)
    st = P.pqnr_inner(n, B, A)
    rows, _ = _sample_rows(X, n, rng, k_random=10)
    Bo, ost = oracle.pqnr_inner(X, n, Bh, M.factors, lmax=8, tau=1e-6, rows=rows)
    got = host(B)
    for i in rows:
        assert_parity(got[i:i + 1], Bo[i:i + 1], 1e-10, f"PQNR row {i}", elementwise=False)
    assert st["inner_iters"] >= ost["n_updates"]
    P.close()


def test_pdnr_inner_fullsize_sampled_rows(big):
    """PDNR row solves of mode 0 at full size (the Hessian pass over 20M
    nonzeros, rows spanning many ranges); the oracle solves the sampled rows
    alone. Gate: the damped solve's condition-number bound after four steps
    at R = 16 (tests/test_gpu_pdnr.py derives it), 1.1e-10."""
    from tests.test_gpu_pdnr import _lockstep_tol
    X, M, sched = big
    lmax = 4
    P = cpapr.Plan.from_tensor(X, M.rank, method=cpapr.CPAPR_METHOD_PDNR, lmax=lmax, tol=1e-6)
    A = [dev(a) for a in M.factors]
    rng = np.random.default_rng(3)
    n = 0
    Bh = M.factors[n] * M.lam
    B = dev(Bh)
    st = P.pdnr_inner(n, B, A)
    rows, _ = _sample_rows(X, n, rng, k_random=10)
    Bo, ost = oracle.pdnr_inner(X, n, Bh, M.factors, lmax=lmax, tau=1e-6, rows=rows)
    got = host(B)
    tol = _lockstep_tol(M.rank, lmax)
    for i in rows:
        assert_parity(got[i:i + 1], Bo[i:i + 1], tol, f"PDNR row {i}", elementwise=False)
    assert st["inner_iters"] >= ost["n_updates"]
    P.close()
