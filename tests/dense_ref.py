"""Dense brute force for tiny tensors: explicit mode-n matricization and
Khatri-Rao product, written independently of the sparse oracle.

Phi(n) = (X_(n) ./ max(B Pi, eps)) Pi^T with Pi = (A(N) (.) ... A(n+1) (.) A(n-1)
(.) ... A(1))^T, the R x J_n matrix of Algorithm 1 and Algorithm 2. The
unfolding is the Kolda-Bader one: among the remaining modes the earlier mode
index varies fastest along the columns, matching the Khatri-Rao order above.
"""
import numpy as np


def densify(X):
    T = np.zeros(X.dims)
    np.add.at(T, tuple(X.idx.astype(np.int64)), X.vals)
    return T


def unfold(T, n):
    return np.reshape(np.moveaxis(T, n, 0), (T.shape[n], -1), order="F")


def khatri_rao(mats):
    """Columnwise Kronecker product of mats[0] (.) mats[1] (.) ...; the last varies fastest."""
    R = mats[0].shape[1]
    out = mats[0]
    for M in mats[1:]:
        out = np.einsum("ir,jr->ijr", out, M).reshape(-1, R)
    return out


def pi_matrix(factors, n):
    others = [factors[m] for m in reversed(range(len(factors))) if m != n]
    return khatri_rao(others).T  # R x J_n


def phi_dense(X, n, B, factors, eps):
    Xn = unfold(densify(X), n)
    Pi = pi_matrix(factors, n)
    D = np.maximum(B @ Pi, eps)
    return (Xn / D) @ Pi.T


def full_model(lam, factors):
    """Dense tensor sum_r lam_r a1_r o a2_r o ... (outer products)."""
    R = lam.shape[0]
    T = np.zeros(tuple(a.shape[0] for a in factors))
    for r in range(R):
        t = np.array(lam[r])
        for a in factors:
            t = np.multiply.outer(t, a[:, r])
        T += t
    return T


def loglik_dense(X, lam, factors):
    """Poisson log-likelihood over every cell, minus the log(x!) constant."""
    T = densify(X)
    M = full_model(lam, factors)
    nz = T > 0
    return float(np.sum(T[nz] * np.log(M[nz])) - np.sum(M))


def mttkrp_dense(X, n, factors):
    return unfold(densify(X), n) @ pi_matrix(factors, n).T
