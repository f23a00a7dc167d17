"""Pins for the FP64 oracle against facts fixed by the paper and by the mathematics,
not by the oracle's own code: dense brute force (explicit matricization and
Khatri-Rao, Algorithm 2), closed forms, exact identities, invariances, the
N = 2 reduction to Lee-Seung KL-NMF, likelihood monotonicity, and recovery of a
planted model. Each pin is chosen so that a plausible slip in the oracle
(a dropped term, a wrong index or sign, a transposed operand, a missing clamp)
fails at least one of them."""
import itertools
import math
import os

import numpy as np
import pytest

from paper_2307_03276_amd import synth
from tests import dense_ref

pytestmark = pytest.mark.usefixtures("oracle_lib")


def tiny_case(seed, dims, nnz, R, distinct=False):
    X = synth.random_tensor(seed, dims, nnz, mu=2.0, distinct=distinct)
    M = synth.random_model(seed, dims, R)
    return X, M


# ---------------------------------------------------------------- Phi (Algorithm 2)

@pytest.mark.parametrize("dims,R", [((5, 4), 3), ((5, 4, 3), 3), ((3, 4, 2, 3), 2),
                                    ((2, 3, 2, 3, 2), 4), ((6, 5, 4), 1)])
def test_phi_matches_dense_bruteforce(oracle_lib, dims, R):
    X, M = tiny_case(11, dims, max(3, math.prod(dims) // 3), R)
    for n in range(len(dims)):
        B = M.factors[n] * M.lam
        got = oracle_lib.phi(X, n, B, M.factors, eps=1e-10)
        ref = dense_ref.phi_dense(X, n, B, M.factors, 1e-10)
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-300)


def test_phi_clamp_matches_dense(oracle_lib):
    """With eps larger than some entries of B Pi the clamp decides the divisor."""
    X, M = tiny_case(3, (4, 5, 3), 25, 2)
    B = M.factors[0] * M.lam * 1e-3
    eps = float(np.median((B @ dense_ref.pi_matrix(M.factors, 0))))
    got = oracle_lib.phi(X, 0, B, M.factors, eps=eps)
    ref = dense_ref.phi_dense(X, 0, B, M.factors, eps)
    np.testing.assert_allclose(got, ref, rtol=1e-13)
    # and the clamp is really active for some nonzero
    Pi = dense_ref.pi_matrix(M.factors, 0)
    assert np.any((B @ Pi)[dense_ref.unfold(dense_ref.densify(X), 0) > 0] < eps)


def test_phi_mass_identity(oracle_lib):
    """sum_{i,r} B[i,r] Phi[i,r] = sum_k x_k when no clamp is active: each nonzero
    contributes s_k * sum_r B[i,r] pi_k[r] = x_k."""
    X = synth.random_tensor(5, (300, 200, 100), 50_000, zipf=(1.1, None, 1.2), mu=3.0)
    M = synth.random_model(5, X.dims, 7)
    for n in range(3):
        B = M.factors[n] * M.lam
        P = oracle_lib.phi(X, n, B, M.factors)
        assert abs(np.sum(B * P) - X.vals.sum()) <= 1e-12 * X.vals.sum()


def test_phi_rank_one_closed_form(oracle_lib):
    """R = 1: Phi[i] = (sum of x_k in row i) / b_i, independent of the other factors."""
    X = synth.random_tensor(8, (50, 40, 30), 3000, zipf=(1.1, 1.1, None))
    M = synth.random_model(8, X.dims, 1)
    for n in range(3):
        B = M.factors[n] * M.lam
        P = oracle_lib.phi(X, n, B, M.factors)
        marg = np.bincount(X.idx[n], weights=X.vals, minlength=X.dims[n])
        np.testing.assert_allclose(P[:, 0], marg / B[:, 0], rtol=1e-13)


def test_phi_scale_invariances(oracle_lib):
    """Phi(B, c*Pi) = Phi(B, Pi) and Phi(c*B, Pi) = Phi(B, Pi)/c (no clamp active)."""
    X, M = tiny_case(21, (30, 20, 10), 800, 5)
    B = M.factors[1] * M.lam
    base = oracle_lib.phi(X, 1, B, M.factors)
    f2 = [a.copy() for a in M.factors]
    f2[2] = f2[2] * 4.0  # scales every pi_k (mode 1's Pi uses modes 0 and 2)
    np.testing.assert_allclose(oracle_lib.phi(X, 1, B, f2), base, rtol=1e-14)
    np.testing.assert_allclose(oracle_lib.phi(X, 1, 8.0 * B, M.factors), base / 8.0, rtol=1e-14)
    # scaling the mode's own factor does not enter Phi (only B does)
    f3 = [a.copy() for a in M.factors]
    f3[1] = f3[1] * 3.0
    np.testing.assert_array_equal(oracle_lib.phi(X, 1, B, f3), base)


def test_phi_order_and_duplicate_invariance(oracle_lib):
    X = synth.random_tensor(4, (20, 15, 10), 4000, zipf=(1.1, 1.1, 1.1))
    M = synth.random_model(4, X.dims, 6)
    B = M.factors[2] * M.lam
    base = oracle_lib.phi(X, 2, B, M.factors)
    perm = np.random.default_rng(0).permutation(X.nnz)
    Xp = synth.SparseTensor(X.dims, np.ascontiguousarray(X.idx[:, perm]), X.vals[perm].copy())
    np.testing.assert_allclose(oracle_lib.phi(Xp, 2, B, M.factors), base, rtol=1e-15)
    # coalesce duplicates: Phi is linear in x, so the coalesced tensor gives the same Phi
    lin = np.ravel_multi_index(tuple(X.idx.astype(np.int64)), X.dims)
    u, inv = np.unique(lin, return_inverse=True)
    assert u.size < X.nnz  # the Zipf draw really produced duplicates
    vals = np.bincount(inv, weights=X.vals)
    Xc = synth.SparseTensor(X.dims, np.stack(np.unravel_index(u, X.dims)).astype(np.int32), vals)
    np.testing.assert_allclose(oracle_lib.phi(Xc, 2, B, M.factors), base, rtol=1e-14)


def test_phi_empty_rows_and_clamped_contribution(oracle_lib):
    dims = (6, 3, 2)
    idx = np.array([[0, 0, 3], [1, 2, 0], [1, 0, 1]], dtype=np.int32)
    vals = np.array([2.0, 5.0, 7.0])
    X = synth.SparseTensor(dims, idx, vals)
    rng = np.random.default_rng(1)
    A = [rng.random((d, 2)) + 0.1 for d in dims]
    B = rng.random((6, 2)) + 0.1
    B[3] = 1e-30  # row 3's only nonzero is clamped: contributes (x/eps) * pi
    eps = 1e-10
    P = oracle_lib.phi(X, 0, B, A, eps=eps)
    for i in (1, 2, 4, 5):
        assert np.all(P[i] == 0.0)
    pi3 = A[1][0] * A[2][1]
    np.testing.assert_allclose(P[3], (7.0 / eps) * pi3, rtol=1e-15)
    # row 0 by hand: two nonzeros
    want = np.zeros(2)
    for k in (0, 1):
        pi = A[1][idx[1, k]] * A[2][idx[2, k]]
        want += vals[k] / max(B[0] @ pi, eps) * pi
    np.testing.assert_allclose(P[0], want, rtol=1e-15)


def test_phi_golden_hand_example(oracle_lib):
    """Hand-worked 2x2x2 example stored under tests/golden (exact rational arithmetic)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "phi_hand_2x2x2.txt")
    sec = _read_golden(path)
    dims = tuple(int(v) for v in sec["dims"][0])
    idx = np.array(sec["idx"], dtype=np.int32).T.copy()
    vals = np.array([r[0] for r in sec["vals"]])
    X = synth.SparseTensor(dims, idx, vals)
    A = [np.array(sec[f"A{m}"]) for m in range(3)]
    B = np.array(sec["B"])
    P = oracle_lib.phi(X, 0, B, A, eps=1e-10)
    np.testing.assert_allclose(P, np.array(sec["Phi0"]), rtol=1e-15)


def _read_golden(path):
    sec, cur = {}, None
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("[") and line.endswith("]"):
                cur = line[1:-1]
                sec[cur] = []
            else:
                sec[cur].append([float(_frac(t)) for t in line.split()])
    return sec


def _frac(t):
    if "/" in t:
        a, b = t.split("/")
        return float(a) / float(b)
    return float(t)


# ---------------------------------------------------------------- MU inner loop (Algorithm 1)

def _ll_mode(X, n, B, factors):
    """Poisson LL of the model [1; A(1).. B (mode n) ..A(N)] by dense brute force."""
    f = [a for a in factors]
    f = f[:n] + [B] + f[n + 1:]
    return dense_ref.loglik_dense(X, np.ones(B.shape[1]), f)


def test_mu_inner_monotone_nonnegative_and_mass(oracle_lib):
    X, M = tiny_case(31, (8, 7, 6), 120, 3)
    for n in range(3):
        B = M.factors[n] * M.lam
        prev = _ll_mode(X, n, B, M.factors)
        for _ in range(6):
            B2, P, hist, nup = oracle_lib.mu_inner(X, n, B, M.factors, lmax=1)
            assert nup == 1
            assert np.all(B2 >= 0) and np.all(P >= 0)
            # mass after the update equals sum x (other columns have unit 1-norm)
            assert abs(B2.sum() - X.vals.sum()) <= 1e-12 * X.vals.sum()
            cur = _ll_mode(X, n, B2, M.factors)
            assert cur >= prev - 1e-10 * abs(prev)
            prev, B = cur, B2


def test_mu_inner_n2_is_lee_seung_kl_nmf(oracle_lib):
    """N = 2: V ~ W H with H = A(2)^T (rows sum to one); the CP-APR MU step for
    B = W is Lee & Seung's KL update W <- W .* ((V ./ (W H)) H^T) ./ (1 H^T)."""
    X, M = tiny_case(41, (9, 7), 40, 3)
    V = dense_ref.densify(X)
    W = M.factors[0] * M.lam
    H = M.factors[1].T
    for _ in range(5):
        W = W * (((V / (W @ H)) @ H.T) / H.sum(axis=1)[None, :])
    B, _, _, nup = oracle_lib.mu_inner(X, 0, M.factors[0] * M.lam, M.factors, lmax=5)
    assert nup == 5
    np.testing.assert_allclose(B, W, rtol=1e-12)


def test_mu_inner_kkt_break(oracle_lib):
    """The KKT test runs before each update: with tau above the first violation
    nothing is updated; the recorded violation is max |min(B, 1 - Phi)|."""
    X, M = tiny_case(51, (10, 8, 6), 200, 3)
    B = M.factors[0] * M.lam
    _, P0, hist, _ = oracle_lib.mu_inner(X, 0, B, M.factors, lmax=1)
    v0 = np.max(np.abs(np.minimum(B, 1 - P0)))
    assert hist[0] == v0
    B2, _, hist2, nup = oracle_lib.mu_inner(X, 0, B, M.factors, lmax=4, tau=v0 * 1.0001)
    assert nup == 0 and np.array_equal(B2, B)
    B3, _, hist3, nup3 = oracle_lib.mu_inner(X, 0, B, M.factors, lmax=4, tau=v0 * 0.9999)
    assert nup3 >= 1


def test_mu_inner_row_restriction_is_exact(oracle_lib):
    X, M = tiny_case(52, (40, 30, 20), 3000, 4)
    B = M.factors[1] * M.lam
    Bf, Pf, _, _ = oracle_lib.mu_inner(X, 1, B, M.factors, lmax=3)
    rows = np.array([0, 5, 17, 29])
    Br, Pr, _, _ = oracle_lib.mu_inner(X, 1, B, M.factors, lmax=3, rows=rows)
    np.testing.assert_array_equal(Br[rows], Bf[rows])
    np.testing.assert_array_equal(Pr[rows], Pf[rows])


# ---------------------------------------------------------------- full solve (Algorithm 1)

def test_solve_rank_one_closed_form(oracle_lib):
    """R = 1: after the first outer iteration the model is the rank-one Poisson MLE
    lambda = sum x, A(n) = mode-n marginal / sum x; at k = 2 the KKT violation is 0,
    so with tau > 0 the solve stops there."""
    X = synth.random_tensor(61, (30, 20, 10), 1500, zipf=(1.1, None, 1.1))
    M = synth.random_model(61, X.dims, 1)
    out, st = oracle_lib.solve(X, M, kmax=1, lmax=3)
    tot = X.vals.sum()
    np.testing.assert_allclose(out.lam, [tot], rtol=1e-13)
    for n in range(3):
        marg = np.bincount(X.idx[n], weights=X.vals, minlength=X.dims[n])
        np.testing.assert_allclose(out.factors[n][:, 0], marg / tot, rtol=1e-12, atol=1e-300)
    out2, st2 = oracle_lib.solve(X, M, kmax=5, lmax=3, tau=1e-8)
    assert st2["converged"] and st2["outer_iters"] == 2


def test_solve_mass_and_normalisation(oracle_lib):
    X, M = tiny_case(71, (25, 20, 15, 4), 1500, 4)
    out, st = oracle_lib.solve(X, M, kmax=3, lmax=4)
    assert abs(out.lam.sum() - X.vals.sum()) <= 1e-12 * X.vals.sum()
    for a in out.factors:
        assert np.all(a >= 0)
        np.testing.assert_allclose(a.sum(axis=0), 1.0, rtol=1e-13)
    assert st["outer_iters"] == 3 and st["inner_updates"] == 3 * 4 * 4


def test_solve_loglik_nondecreasing(oracle_lib):
    X, M = tiny_case(72, (20, 15, 10), 600, 3)
    prev = oracle_lib.loglik(X, M)
    cur = M
    for _ in range(4):
        cur, _ = oracle_lib.solve(X, cur, kmax=1, lmax=5)
        ll = oracle_lib.loglik(X, cur)
        assert ll >= prev - 1e-10 * abs(prev)
        prev = ll


def test_solve_inadmissible_zero_shift(oracle_lib):
    """MU alone never moves an exact zero (B .* Phi); S lifts a zero entry whose
    previous Phi exceeds 1, from the second outer iteration on, and only such
    entries: an admissible zero (Phi <= 1) and an empty row stay exactly zero,
    and a model without tiny entries is unaffected by kappa."""
    X, M = tiny_case(81, (12, 10, 8), 400, 3)
    keep = X.idx[0] != 11  # row 11 of mode 0 is made empty: its Phi stays 0
    # row 5 of mode 0 only meets mode-1 coordinate 0, whose component-2 weight is tiny,
    # so Phi(mode 0)[5, 2] << 1 in the first sweep: an admissible zero
    keep &= (X.idx[0] != 5) | (X.idx[1] == 0)
    X = synth.SparseTensor(X.dims, np.ascontiguousarray(X.idx[:, keep]), X.vals[keep].copy())
    assert np.any(X.idx[0] == 5)
    base = M.copy()
    M.factors[1][0, 2] = 1e-9
    M.factors[0][2, 1] = 0.0  # row 2 has nonzeros: Phi[2,1] > 1 once the model fits
    M.factors[0][11, 0] = 0.0
    M.factors[0][5, 2] = 0.0
    noS, _ = oracle_lib.solve(X, M, kmax=4, lmax=3, kappa=0.0)
    assert noS.factors[0][2, 1] == 0.0
    withS, _ = oracle_lib.solve(X, M, kmax=4, lmax=3, kappa=0.01)
    assert withS.factors[0][2, 1] > 0.0
    assert withS.factors[0][11, 0] == 0.0
    two, _ = oracle_lib.solve(X, M, kmax=2, lmax=3, kappa=0.01)
    assert two.factors[0][5, 2] == 0.0
    one, _ = oracle_lib.solve(X, M, kmax=1, lmax=3, kappa=0.01)
    assert one.factors[0][2, 1] == 0.0  # no shift in the first outer iteration
    # no entry below kappa_tol: kappa changes nothing
    a, _ = oracle_lib.solve(X, base, kmax=3, lmax=3, kappa=0.0)
    b, _ = oracle_lib.solve(X, base, kmax=3, lmax=3, kappa=0.5)
    for fa, fb in zip(a.factors, b.factors):
        assert np.array_equal(fa, fb)


def test_loglik_matches_dense(oracle_lib):
    X, M = tiny_case(91, (6, 5, 4), 40, 3)
    np.testing.assert_allclose(oracle_lib.loglik(X, M), dense_ref.loglik_dense(X, M.lam, M.factors),
                               rtol=1e-13)


def test_solve_planted_recovery(oracle_lib):
    """Sparse nonnegative planted model, X ~ Poisson(M_true) densely sampled;
    the best of three seeded fits recovers the components (factor match score)."""
    rng = np.random.default_rng(2024)
    dims, R = (40, 30, 20), 3
    facs = []
    for d in dims:
        a = np.zeros((d, R))
        for r in range(R):
            sup = rng.choice(d, size=max(3, d // 4), replace=False)
            a[sup, r] = rng.random(sup.size) + 0.2
        facs.append(a / a.sum(axis=0))
    lam = np.array([2000.0, 1500.0, 1000.0])
    T = rng.poisson(dense_ref.full_model(lam, facs))
    nzi = np.nonzero(T)
    X = synth.SparseTensor(dims, np.stack(nzi).astype(np.int32), T[nzi].astype(np.float64))
    best, best_ll = None, -np.inf
    for s in range(3):
        M0 = synth.random_model(100 + s, dims, R)
        out, _ = oracle_lib.solve(X, M0, kmax=200, lmax=10, tau=1e-4)
        ll = oracle_lib.loglik(X, out)
        if ll > best_ll:
            best, best_ll = out, ll
    score = 0.0
    for perm in itertools.permutations(range(R)):
        per_comp = []
        for r in range(R):
            c = 1.0
            for n in range(3):
                u, v = facs[n][:, r], best.factors[n][:, perm[r]]
                c *= (u @ v) / (np.linalg.norm(u) * np.linalg.norm(v))
            per_comp.append(c)
        score = max(score, float(np.mean(per_comp)))
    assert score >= 0.9


# ---------------------------------------------------------------- MTTKRP (Eqs. 10-12)

@pytest.mark.parametrize("dims", [(5, 4, 3), (3, 4, 2, 3)])
def test_mttkrp_matches_dense(oracle_lib, dims):
    X, M = tiny_case(99, dims, 20, 3)
    for n in range(len(dims)):
        np.testing.assert_allclose(oracle_lib.mttkrp(X, n, M.factors),
                                   dense_ref.mttkrp_dense(X, n, M.factors), rtol=1e-13)
