"""Parity at the largest single-GPU size: the 4-way 1M x 200k x 10k x 500 tensor
with 100M nonzeros (Zipf(1.2) on modes 1-2, uniform on 3-4, counts capped at
1000), R = 32, in the default launch shape (the launch-policy model's: 16 lanes x 2 rank
columns in FP64, 8 lanes x 4 with FP32-stored factors).

As at 20M: oracle rows one by one (Phi and the fixed-schedule inner loop are
row-separable), plus the mass identity sum(B .* Phi) = sum(x) over every row.
The heaviest row of modes 1-2 holds about a fifth of all nonzeros, so it spans
thousands of tiles and exercises the tile-boundary merges at full size."""
import numpy as np
import pytest

import oracle
from paper_2307_03276_amd import cpapr, synth
from tests.gpu_util import assert_parity, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big4():
    import torch
    assert torch.cuda.is_available()
    oracle.build(force=False)
    print("generating the 4-way 100M-nonzero tensor", flush=True)
    X, M, sched = synth.config_zipf4()
    return X, M, sched


def _sample_rows(X, n, rng, k_random=16):
    counts = np.bincount(X.idx[n], minlength=X.dims[n])
    heavy = np.argsort(counts)[-4:]
    nonempty = np.flatnonzero(counts)
    empty = np.flatnonzero(counts == 0)
    pick = [heavy, rng.choice(nonempty, size=min(k_random, nonempty.size), replace=False)]
    if empty.size:
        pick.append(rng.choice(empty, size=min(4, empty.size), replace=False))
    return np.unique(np.concatenate(pick)), counts


@pytest.mark.parametrize("precision,tol", [(cpapr.CPAPR_FP64, 1e-12), (cpapr.CPAPR_MIXED, 1e-5)])
def test_phi_4way_fullsize_sampled_rows_and_mass(big4, precision, tol):
    X, M, sched = big4
    P = cpapr.Plan.from_tensor(X, M.rank, precision=precision, lmax=sched["lmax"], tol=0.0)
    A = [dev(a) for a in M.factors]
    rng = np.random.default_rng(0)
    total = X.vals.sum()
    for n in range(4):
        Bh = M.factors[n] * M.lam
        got = host(P.phi(n, dev(Bh), A))
        rows, counts = _sample_rows(X, n, rng)
        ref = oracle.phi(X, n, Bh, M.factors, rows=rows)
        assert_parity(got[rows], ref[rows], tol, f"mode {n} sampled rows")
        mass = float(np.sum(Bh * got))
        assert abs(mass - total) <= tol * total, f"mode {n} mass {mass} vs {total}"
        assert np.all(got[counts == 0] == 0)
    P.close()


def test_mttkrp_4way_fullsize_sampled_rows(big4):
    """MTTKRP at the 100M-nonzero size in the benchmarked launch shape:
    sampled rows (one heavy row and random ones) against the oracle, which
    computes them from those rows' nonzeros; empty rows exactly zero."""
    X, M, _ = big4
    P = cpapr.Plan.from_tensor(X, M.rank)
    A = [dev(a) for a in M.factors]
    rng = np.random.default_rng(4)
    for n in range(4):
        got = host(P.mttkrp(n, A))
        counts = np.bincount(X.idx[n], minlength=X.dims[n])
        nonempty = np.flatnonzero(counts)
        rows = np.unique(np.concatenate([[np.argmax(counts)],
                                         rng.choice(nonempty, size=min(12, nonempty.size), replace=False)]))
        sel = np.isin(X.idx[n], rows)
        Xs = synth.SparseTensor(X.dims, np.ascontiguousarray(X.idx[:, sel]), X.vals[sel].copy())
        ref = oracle.mttkrp(Xs, n, M.factors)[rows]
        assert_parity(got[rows], ref, 1e-12, f"MTTKRP mode {n} sampled rows")
        assert np.all(got[counts == 0] == 0)
    P.close()


def test_mu_inner_4way_fullsize_sampled_rows(big4):
    X, M, sched = big4
    P = cpapr.Plan.from_tensor(X, M.rank, lmax=sched["lmax"], tol=0.0)
    A = [dev(a) for a in M.factors]
    rng = np.random.default_rng(1)
    n = 1
    Bh = M.factors[n] * M.lam
    B = dev(Bh)
    phi_last, st = P.mu_inner(n, B, A)
    assert st["inner_iters"] == sched["lmax"] and st["phi_evals"] == sched["lmax"]
    rows, _ = _sample_rows(X, n, rng, k_random=8)
    Bo, Po, _, _ = oracle.mu_inner(X, n, Bh, M.factors, lmax=sched["lmax"], rows=rows)
    assert_parity(host(B)[rows], Bo[rows], 1e-12, "B rows")
    assert_parity(host(phi_last)[rows], Po[rows], 1e-12, "Phi rows")
    P.close()
