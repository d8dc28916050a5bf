"""Residual-correlation neighbors for VIF (oracle; test infrastructure only).

In the VIF approximation the Vecchia factor is built on the residual of the
low-rank part (Sec. "The Vecchia-inducing-point full-scale approximation"), and
the paper's VIF selects that factor's conditioning sets by correlation of the
residual process (the correlation metric of Sec. "Correlation-based Vecchia
neighbor selection" applied to the residual covariance, as done for VIF by the
work it builds on). With U = C(X,Z) L_k^-T:

    r(p, q) = C(p, q) - U_p . U_q          (latent residual; the nugget is
                                            excluded, as for the plain search)
    rho(i, j) = |r(i, j)| / sqrt(r(i, i) r(j, j)).

For query i the ranking over j < i by rho descending equals the ranking by
    key(i, j) = r(i, j)^2 / r(j, j)
(r(i, i) is common to the row). A candidate whose residual variance r(j, j)
is not positive (a point the inducing points explain completely) gets key -1,
after every other candidate. Ties go to the lower index; row i holds the first
min(i, m) candidates, padded with -1. This is the plain definition written out
(a brute-force top-m); it is not fast.
"""
from __future__ import annotations

import numpy as np

from .kernels import cov
from .likelihood import low_rank_factor, low_rank_rows


def residual_parts(kern, X, Z, jitter=0.0):
    """U [n, k] and the residual variances r(j, j) [n]."""
    sx = X[0]
    n = sx.shape[0]
    if Z is None or Z[0].shape[0] == 0:
        U = np.zeros((n, 0))
    else:
        Lk = low_rank_factor(kern, Z, jitter)
        U = low_rank_rows(kern, X, Z, Lk, np.arange(n))
    d = kern["sigma2"] - (U * U).sum(1)
    return U, d


def row_keys(kern, X, U, d, i, js):
    """key(i, j) for the candidates js of query i."""
    sx, sy, t = X
    js = np.asarray(js, dtype=np.int64)
    c = cov(kern, sx[i] - sx[js], sy[i] - sy[js], t[i] - t[js])
    r = c - U[js] @ U[i]
    dj = d[js]
    out = np.full(js.shape[0], -1.0)
    pos = dj > 0
    out[pos] = r[pos] * r[pos] / dj[pos]
    return out


def brute_force(kern, X, Z, m, rows=None, jitter=0.0):
    """Residual-correlation neighbor rows [len(rows), m] (-1 padded)."""
    n = X[0].shape[0]
    U, d = residual_parts(kern, X, Z, jitter)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    out = np.full((rows.shape[0], m), -1, dtype=np.int32)
    for r, i in enumerate(rows):
        if i == 0 or m == 0:
            continue
        js = np.arange(i)
        k = row_keys(kern, X, U, d, i, js)
        order = np.lexsort((js, -k))[:m]
        out[r, :order.shape[0]] = js[order]
    return out
