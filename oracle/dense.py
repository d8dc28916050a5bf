"""Dense FP64 likelihoods used only to pin the oracle (test infrastructure only).

* exact      -- the Gaussian NLL of Sec. "Estimation and prediction" by a dense
                Cholesky of Sigma + nugget I;
* fitc       -- the FITC covariance of Sec. "Low-rank inducing point
                approximations" (low rank plus diagonal correction) with the
                nugget added, by dense Cholesky;
* vif_dense  -- the VIF covariance U U' + B^-1 D B^-T assembled as a dense n x n
                matrix from a factor (A, D), by dense Cholesky; checks the
                Woodbury / determinant-lemma assembly independently;
* kl         -- KL(N(0, S) || N(0, Q^-1)) for a precision Q = B' D^-1 B.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import solve_triangular

from .kernels import cov_matrix

LOG2PI = math.log(2.0 * math.pi)


def gaussian_nll(S, y):
    """n/2 log 2pi + 1/2 log det S + 1/2 y' S^-1 y by dense Cholesky."""
    L = np.linalg.cholesky(S)
    v = solve_triangular(L, y, lower=True)
    return float(0.5 * y.shape[0] * LOG2PI + np.log(np.diag(L)).sum() + 0.5 * v @ v)


def exact_cov(kern, X):
    n = X[0].shape[0]
    return cov_matrix(kern, X, X) + kern["nugget"] * np.eye(n)


def exact_nll(kern, X, y):
    return gaussian_nll(exact_cov(kern, X), y)


def low_rank_dense(kern, X, Z, jitter=0.0):
    """U = C(X,Z) L_k^-T, computed densely with an explicit Sigma_k inverse."""
    k = Z[0].shape[0]
    Skk = cov_matrix(kern, Z, Z) + jitter * np.eye(k)
    Ckn = cov_matrix(kern, Z, X)
    Lk = np.linalg.cholesky(Skk)
    return solve_triangular(Lk, Ckn, lower=True).T


def fitc_nll(kern, X, y, Z, jitter=0.0):
    U = low_rank_dense(kern, X, Z, jitter)
    diag = kern["sigma2"] + kern["nugget"] - (U * U).sum(1)
    return gaussian_nll(U @ U.T + np.diag(diag), y)


def b_matrix(A, nbr):
    """Dense unit lower-triangular B with B[i, N(i)] = -A_i."""
    n, m = nbr.shape
    B = np.eye(n)
    for i in range(n):
        for r in range(m):
            j = nbr[i, r]
            if j >= 0:
                B[i, j] = -A[i, r]
    return B


def vecchia_cov(A, D, nbr):
    """B^-1 D B^-T."""
    B = b_matrix(A, nbr)
    Binv = solve_triangular(B, np.eye(B.shape[0]), lower=True, unit_diagonal=True)
    return Binv @ np.diag(D) @ Binv.T


def vif_dense_nll(kern, X, y, A, D, nbr, Z, jitter=0.0):
    U = low_rank_dense(kern, X, Z, jitter) if Z[0].shape[0] else np.zeros((X[0].shape[0], 0))
    return gaussian_nll(U @ U.T + vecchia_cov(A, D, nbr), y)


def kl_gauss(S, A, D, nbr):
    """KL(N(0,S) || N(0, B^-1 D B^-T)) = 1/2 [tr(Q S) - n + log det(Q^-1) - log det S]."""
    B = b_matrix(A, nbr)
    Q = B.T @ np.diag(1.0 / D) @ B
    n = S.shape[0]
    L = np.linalg.cholesky(S)
    return float(0.5 * (np.trace(Q @ S) - n + np.log(D).sum() - 2.0 * np.log(np.diag(L)).sum()))
