"""Property-based pins of the oracle (hypothesis): random small shapes, ranks,
value scales and floors against the dense definitions written out in NumPy
(explicit unfolding and Khatri-Rao products), and the identities that hold for
any input."""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from paper_2307_03276_amd import synth
from tests import dense_ref

pytestmark = pytest.mark.usefixtures("oracle_lib")

shapes = st.lists(st.integers(1, 5), min_size=2, max_size=5).filter(lambda d: math.prod(d) <= 400)
cfg = settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])


@cfg
@given(dims=shapes, R=st.integers(1, 6), seed=st.integers(0, 10_000), scale=st.sampled_from([1e-6, 1.0, 1e6]),
       eps=st.sampled_from([1e-10, 1e-3]))
def test_phi_equals_dense_definition(oracle_lib, dims, R, seed, scale, eps):
    dims = tuple(dims)
    nnz = max(1, math.prod(dims) // 2)
    X = synth.random_tensor(seed, dims, nnz)
    M = synth.random_model(seed, dims, R)
    for n in range(len(dims)):
        B = M.factors[n] * M.lam * scale
        got = oracle_lib.phi(X, n, B, M.factors, eps=eps)
        ref = dense_ref.phi_dense(X, n, B, M.factors, eps)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-300)


@cfg
@given(dims=shapes, R=st.integers(1, 5), seed=st.integers(0, 10_000))
def test_mass_identity_and_mttkrp_definition(oracle_lib, dims, R, seed):
    """sum(B .* Phi) = sum(x) whenever no model value is clamped; MTTKRP is the
    unfolding times the Khatri-Rao product."""
    dims = tuple(dims)
    X = synth.random_tensor(seed, dims, max(1, math.prod(dims) // 2))
    M = synth.random_model(seed, dims, R)
    for n in range(len(dims)):
        B = M.factors[n] * M.lam
        phi = oracle_lib.phi(X, n, B, M.factors)
        assert abs(np.sum(B * phi) - X.vals.sum()) <= 1e-12 * X.vals.sum()
        np.testing.assert_allclose(oracle_lib.mttkrp(X, n, M.factors), dense_ref.mttkrp_dense(X, n, M.factors),
                                   rtol=1e-12, atol=1e-300)


@cfg
@given(dims=shapes, R=st.integers(1, 5), seed=st.integers(0, 10_000))
def test_loglik_equals_dense_definition(oracle_lib, dims, R, seed):
    dims = tuple(dims)
    X = synth.random_tensor(seed, dims, max(1, math.prod(dims) // 2))
    M = synth.random_model(seed, dims, R)
    ref = dense_ref.loglik_dense(X, M.lam, M.factors)
    assert abs(oracle_lib.loglik(X, M) - ref) <= 1e-12 * max(1.0, abs(ref))


def _row_objective(X, n, B, factors, eps=1e-10):
    """Sum over rows of f_i(b) = sum(b) - sum_k x_k log(max(b . pi_k, eps)), in NumPy."""
    pi = np.ones((X.nnz, B.shape[1]))
    for m in range(X.nmodes):
        if m != n:
            pi *= factors[m][X.idx[m]]
    mk = np.einsum("kr,kr->k", B[X.idx[n]], pi)
    return float(B.sum() - np.sum(X.vals * np.log(np.maximum(mk, eps))))


@cfg
@given(dims=shapes, R=st.integers(1, 5), seed=st.integers(0, 10_000), lmax=st.integers(1, 6))
def test_row_solvers_descend_and_stay_feasible(oracle_lib, dims, R, seed, lmax):
    """PQNR and PDNR never increase the row objectives, keep B >= 0 and report
    the steps they took (lmax per row on a fixed schedule)."""
    dims = tuple(dims)
    X = synth.random_tensor(seed, dims, max(1, math.prod(dims) // 2))
    M = synth.random_model(seed, dims, R)
    for n in range(len(dims)):
        B0 = M.factors[n] * M.lam
        f0 = _row_objective(X, n, B0, M.factors)
        for solve in (oracle_lib.pqnr_inner, oracle_lib.pdnr_inner):
            B, st_ = solve(X, n, B0, M.factors, lmax=lmax, tau=0.0)
            assert np.all(B >= 0)
            assert _row_objective(X, n, B, M.factors) <= f0 + 1e-12 * abs(f0)
            assert st_["n_updates"] == lmax and st_["row_steps"] == lmax * X.dims[n]
