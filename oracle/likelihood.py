"""Vecchia and VIF negative log-likelihoods in FP64 (oracle; test infrastructure only).

Negative log-marginal likelihood (Sec. "Estimation and prediction"):
    L = n/2 log(2 pi) + 1/2 log det(Sigma~) + 1/2 y' Sigma~^-1 y,
    Sigma~ = Sigma + nugget * I, with y the residual after the mean.

Vecchia (Sec. "Vecchia approximation"): with N(i) the neighbors of i,
    A_i = Sigma_{i,N(i)} Sigma_{N(i)}^-1,   D_i = Sigma_ii - A_i Sigma_{i,N(i)}',
B unit lower-triangular with B_{i,N(i)} = -A_i, so that Cov = B^-1 D B^-T.
Reading: the factor is applied to the response covariance Sigma~ (nugget on the
diagonal of every conditioning block and of Sigma_ii), which gives
    L_V = n/2 log 2pi + 1/2 sum log D_i + 1/2 sum e_i^2 / D_i,
    e_i = y_i - A_i y_N(i).

VIF (Sec. "The Vecchia-inducing-point full-scale approximation"): low-rank part
Sigma_l = Sigma_nk Sigma_k^-1 Sigma_kn = U U' with U = Sigma_nk L_k^-T,
L_k = chol(Sigma_k + jitter I); the Vecchia factor is built on the residual
covariance r~(p,q) = C(p,q) + nugget delta_pq - U_p . U_q (reading: the nugget
is carried by the residual part). With W = D^-1/2 B U and z = D^-1/2 B y the
Woodbury identity and the matrix determinant lemma give
    M = I + W'W,  q = W'z,
    L_VIF = n/2 log 2pi + 1/2 (sum log D_i + log det M) + 1/2 (z'z - q' M^-1 q).
The paper states the resulting cost O(n (m^3 + m^2 k + k^2)) next to the VIF
definition; this oracle does not try to meet it.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import solve_triangular

from .kernels import cov, cov_matrix

LOG2PI = math.log(2.0 * math.pi)


def _pts(d):
    return d[0], d[1], d[2]


def _counts(nbr):
    return (nbr >= 0).sum(1)


def _chunks(rows, per_row_bytes, budget=1 << 28):
    step = max(16, int(budget // max(per_row_bytes, 1)))
    for a in range(0, rows.shape[0], step):
        yield rows[a:a + step]


def low_rank_factor(kern, Z, jitter=0.0):
    """L_k = chol(C(Z,Z) + jitter I), lower triangular, FP64."""
    k = Z[0].shape[0]
    Skk = cov_matrix(kern, Z, Z) + jitter * np.eye(k)
    return np.linalg.cholesky(Skk)


def low_rank_rows(kern, X, Z, Lk, idx):
    """Rows idx of U = C(X,Z) L_k^-T (a triangular solve per column block)."""
    Xi = (X[0][idx], X[1][idx], X[2][idx])
    Ckn = cov_matrix(kern, Z, Xi)
    return solve_triangular(Lk, Ckn, lower=True).T


def vecchia(kern, X, y, nbr):
    """Plain Vecchia factor on the response covariance and its NLL.

    Returns dict with A [n,m] (zeros beyond each row's neighbor count), D, e, nll.
    """
    sx, sy, t = _pts(X)
    n, m = nbr.shape
    s = kern["sigma2"] + kern["nugget"]
    A = np.zeros((n, m))
    D = np.empty(n)
    e = np.empty(n)
    cnt = _counts(nbr)
    for p in np.unique(cnt):
        rows_p = np.nonzero(cnt == p)[0]
        if p == 0:
            D[rows_p] = s
            e[rows_p] = y[rows_p]
            continue
        for rows in _chunks(rows_p, 8 * (p + 1) * (p + 1) * 4):
            N = nbr[rows, :p].astype(np.int64)
            G = cov(kern, sx[N][:, :, None] - sx[N][:, None, :], sy[N][:, :, None] - sy[N][:, None, :],
                    t[N][:, :, None] - t[N][:, None, :])
            G = G + kern["nugget"] * np.eye(p)[None]
            g = cov(kern, sx[N] - sx[rows][:, None], sy[N] - sy[rows][:, None],
                    t[N] - t[rows][:, None])
            Ai = np.linalg.solve(G, g[:, :, None])[:, :, 0]
            A[rows, :p] = Ai
            D[rows] = s - (Ai * g).sum(1)
            e[rows] = y[rows] - (Ai * y[N]).sum(1)
    nll = 0.5 * n * LOG2PI + 0.5 * np.log(D).sum() + 0.5 * (e * e / D).sum()
    return {"A": A, "D": D, "e": e, "nll": float(nll)}


def vif_points(kern, X, y, nbr, Z, Lk, rows, want_w=True):
    """Per-point VIF residual factor for the given rows.

    Returns A [len(rows), m], D, e, z and (optionally) W rows = (U_i - A_i U_N)/sqrt(D_i).
    """
    sx, sy, t = _pts(X)
    m = nbr.shape[1]
    k = Z[0].shape[0]
    rows = np.asarray(rows, dtype=np.int64)
    A = np.zeros((rows.shape[0], m))
    D = np.empty(rows.shape[0])
    e = np.empty(rows.shape[0])
    W = np.empty((rows.shape[0], k)) if want_w else None
    cnt = _counts(nbr[rows])
    nug = kern["nugget"]
    for p in np.unique(cnt):
        sel_p = np.nonzero(cnt == p)[0]
        for sel in _chunks(sel_p, 8 * (p + 1) * (max(k, 1) + (p + 1) * 4)):
            ri = rows[sel]
            N = nbr[ri, :p].astype(np.int64)
            S = np.concatenate([N, ri[:, None]], 1)                 # [B, p+1], i last
            uniq, inv = np.unique(S.reshape(-1), return_inverse=True)
            Uu = low_rank_rows(kern, X, Z, Lk, uniq)                # [u, k]
            US = Uu[inv.reshape(S.shape)]                           # [B, p+1, k]
            C = cov(kern, sx[S][:, :, None] - sx[S][:, None, :], sy[S][:, :, None] - sy[S][:, None, :],
                    t[S][:, :, None] - t[S][:, None, :])
            R = C + nug * np.eye(p + 1)[None] - US @ np.transpose(US, (0, 2, 1))
            rii = R[:, p, p]
            if p == 0:
                Ai = np.zeros((ri.shape[0], 0))
                Di = rii
                ei = y[ri]
            else:
                Ai = np.linalg.solve(R[:, :p, :p], R[:, :p, p][:, :, None])[:, :, 0]
                Di = rii - (Ai * R[:, :p, p]).sum(1)
                ei = y[ri] - (Ai * y[N]).sum(1)
            A[sel, :p] = Ai
            D[sel] = Di
            e[sel] = ei
            if want_w:
                W[sel] = (US[:, p, :] - np.einsum("bp,bpk->bk", Ai, US[:, :p, :])) / np.sqrt(Di)[:, None]
    z = e / np.sqrt(D)
    return {"A": A, "D": D, "e": e, "z": z, "W": W}


def vif(kern, X, y, nbr, Z, jitter=0.0, keep_w=False):
    """VIF factor and NLL. Z=(zx,zy,zt) with k inducing points; k=0 is plain Vecchia."""
    n = X[0].shape[0]
    k = Z[0].shape[0]
    if k == 0:
        out = vecchia(kern, X, y, nbr)
        out["z"] = out["e"] / np.sqrt(out["D"])
        out["logdetM"] = 0.0
        out["quadM"] = 0.0
        return out
    Lk = low_rank_factor(kern, Z, jitter)
    pt = vif_points(kern, X, y, nbr, Z, Lk, np.arange(n), want_w=True)
    W, z, D = pt["W"], pt["z"], pt["D"]
    M = np.eye(k) + W.T @ W
    q = W.T @ z
    LM = np.linalg.cholesky(M)
    logdetM = 2.0 * np.log(np.diag(LM)).sum()
    v = solve_triangular(LM, q, lower=True)
    quad = float(v @ v)
    nll = 0.5 * n * LOG2PI + 0.5 * (np.log(D).sum() + logdetM) + 0.5 * (float(z @ z) - quad)
    out = {"A": pt["A"], "D": D, "e": pt["e"], "z": z, "M": M, "q": q, "Lk": Lk,
           "logdetM": float(logdetM), "quadM": quad, "nll": float(nll),
           "sum_logD": float(np.log(D).sum()), "zz": float(z @ z)}
    if keep_w:
        out["W"] = W
    return out
