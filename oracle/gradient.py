"""Gradient of the Vecchia and VIF NLLs with respect to the kernel
hyperparameters (oracle; test infrastructure only). vecchia_grad works block by
block (below); vif_grad differentiates the VIF covariance in dense form (its
docstring).

The paper fits the hyperparameters by minimising the NLL with a quasi-Newton
method driven by its gradient (Sec. "Estimation and prediction"). For a
Gaussian with covariance Sigma~(theta) the gradient of the NLL is
    d/dtheta = 1/2 tr(Sigma~^-1 dSigma~) - 1/2 alpha' dSigma~ alpha,
    alpha = Sigma~^-1 y.
The Vecchia NLL (on the response covariance, as in the likelihood oracle) is a
sum over points of 1/2 [l(S_i) - l(N_i)] + 1/2 log 2pi, where S_i = N(i) + {i}
and l(T) = log det Sigma~_TT + y_T' Sigma~_TT^-1 y_T (log D_i and e_i^2 / D_i are
such differences), so its gradient is the sum of 1/2 [dl(S_i) - dl(N_i)], each
term the Gaussian formula above on one small block. This module computes
exactly that, block by block, with dense inverses.

Parameters, in this order:
  GNEITING:        sigma2, nugget, a, c, alpha, beta, gamma, tau
  GNEITING_MATERN: sigma2, nugget, a, c, alpha, gamma, delta   (nu fixed)
  MATERN_ANISO:    sigma2, nugget, range_s, range_t   (nu fixed)
The covariance derivatives below follow from the kernel definitions by the
chain rule (psi = a |dt|^(2 alpha) + 1, g = (|ds|^2)^gamma, E = psi^(-beta gamma),
C = sigma2 psi^-tau exp(-c g E); Gneiting-Matern: x = c |ds| psi^(-gamma/2),
C = sigma2 psi^-(delta + gamma) g_nu(x); Matern: C = sigma2 g_nu(d),
d = sqrt(|ds|^2 / range_s^2 + dt^2 / range_t^2)).
"""
from __future__ import annotations

import math

import numpy as np

from .kernels import GNEITING, GNEITING_MATERN, MATERN_ANISO, cov, cov_matrix, matern_closed

LOG2PI = math.log(2.0 * math.pi)

PARAMS = {GNEITING: ("sigma2", "nugget", "a", "c", "alpha", "beta", "gamma", "tau"),
          GNEITING_MATERN: ("sigma2", "nugget", "a", "c", "alpha", "gamma", "delta"),
          MATERN_ANISO: ("sigma2", "nugget", "range_s", "range_t")}


def _matern_dx(nu, x):
    """Derivative of the closed-form Matern correlation g_nu with respect to x."""
    e = np.exp(-x)
    if nu == 0.5:
        return -e
    if nu == 1.5:
        return -x * e
    if nu == 2.5:
        return -x * (1.0 + x) * e / 3.0
    raise ValueError("nu in {0.5, 1.5, 2.5}")


def dcov(kern, dx, dy, dt):
    """Derivatives of the latent covariance, one array per parameter of PARAMS
    (the nugget's is zero: it enters Sigma~ on the diagonal only)."""
    dx, dy, dt = (np.asarray(v, dtype=np.float64) for v in (dx, dy, dt))
    h2 = dx * dx + dy * dy
    C = cov(kern, dx, dy, dt)
    zero = np.zeros_like(C)
    if kern["kind"] == GNEITING:
        a, c, al, be, ga, tau = (kern[k] for k in ("a", "c", "alpha", "beta", "gamma", "tau"))
        adt = np.abs(dt)
        ta = adt ** (2.0 * al)
        psi = a * ta + 1.0
        lp = np.log(psi)
        E = psi ** (-be * ga)
        g = h2 ** ga
        q = c * g * E
        with np.errstate(divide="ignore", invalid="ignore"):
            ldt = np.where(adt > 0, np.log(np.where(adt > 0, adt, 1.0)), 0.0)
            lh2 = np.where(h2 > 0, np.log(np.where(h2 > 0, h2, 1.0)), 0.0)
        dlp = C * (-tau + be * ga * q) / psi          # dC/dpsi
        return [C / kern["sigma2"], zero,
                dlp * ta,                              # a
                -C * g * E,                            # c
                dlp * a * ta * 2.0 * ldt,              # alpha
                C * q * ga * lp,                       # beta
                -C * q * (lh2 - be * lp),              # gamma
                -C * lp]                               # tau
    if kern["kind"] == GNEITING_MATERN:
        a, c, al, ga, de, nu = (kern[k] for k in ("a", "c", "alpha", "gamma", "delta", "nu"))
        adt = np.abs(dt)
        ta = adt ** (2.0 * al)
        psi = a * ta + 1.0
        lp = np.log(psi)
        amp = kern["sigma2"] * psi ** (-(de + ga))     # C = amp g(x)
        x = c * np.sqrt(h2) * psi ** (-ga / 2.0)
        gx = x * _matern_dx(nu, x)                     # x g'(x): dC/dlog x = amp gx
        with np.errstate(divide="ignore", invalid="ignore"):
            ldt = np.where(adt > 0, np.log(np.where(adt > 0, adt, 1.0)), 0.0)
        dpsi = (-(de + ga) * C - 0.5 * ga * amp * gx) / psi   # dC/dpsi
        return [C / kern["sigma2"], zero,
                dpsi * ta,                             # a
                amp * gx / c,                          # c
                dpsi * a * ta * 2.0 * ldt,             # alpha
                -C * lp - 0.5 * amp * gx * lp,         # gamma
                -C * lp]                               # delta
    if kern["kind"] == MATERN_ANISO:
        rs, rt, nu = kern["range_s"], kern["range_t"], kern["nu"]
        d = np.sqrt(h2 / (rs * rs) + dt * dt / (rt * rt))
        e = np.exp(-d)
        if nu == 0.5:
            fp = -e
        elif nu == 1.5:
            fp = -d * e
        elif nu == 2.5:
            fp = -d * (1.0 + d) * e / 3.0
        else:
            raise ValueError("nu in {0.5, 1.5, 2.5}")
        with np.errstate(divide="ignore", invalid="ignore"):
            inv_d = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
        s2 = kern["sigma2"]
        return [C / s2, zero,
                s2 * fp * (-h2 / (rs ** 3)) * inv_d,
                s2 * fp * (-dt * dt / (rt ** 3)) * inv_d]
    raise ValueError("gradient implemented for GNEITING, GNEITING_MATERN and MATERN_ANISO")


def _block(kern, X, idx):
    sx, sy, t = X
    P = len(PARAMS[kern["kind"]])
    dX = sx[idx][:, :, None] - sx[idx][:, None, :]
    dY = sy[idx][:, :, None] - sy[idx][:, None, :]
    dT = t[idx][:, :, None] - t[idx][:, None, :]
    q = idx.shape[1]
    S = cov(kern, dX, dY, dT) + kern["nugget"] * np.eye(q)[None]
    dS = dcov(kern, dX, dY, dT)
    dS[1] = np.broadcast_to(np.eye(q)[None], S.shape).copy()  # nugget
    assert len(dS) == P
    return S, dS


def _dl(S, dS, yv):
    """d l(T) for a batch of blocks: tr(S^-1 dS_p) - alpha' dS_p alpha, [B, P]."""
    if S.shape[1] == 0:
        return np.zeros((S.shape[0], len(dS)))
    Si = np.linalg.inv(S)
    al = np.einsum("bij,bj->bi", Si, yv)
    out = np.empty((S.shape[0], len(dS)))
    for p, D in enumerate(dS):
        out[:, p] = np.einsum("bij,bji->b", Si, D) - np.einsum("bi,bij,bj->b", al, D, al)
    return out


def _l(S, yv):
    if S.shape[1] == 0:
        return np.zeros(S.shape[0])
    _, ld = np.linalg.slogdet(S)
    return ld + np.einsum("bi,bi->b", yv, np.linalg.solve(S, yv[:, :, None])[:, :, 0])


def vecchia_grad(kern, X, y, nbr):
    """(NLL, gradient [P]) of the Vecchia NLL on Sigma + nugget I."""
    n = X[0].shape[0]
    P = len(PARAMS[kern["kind"]])
    cnt = (nbr >= 0).sum(1)
    nll = 0.5 * n * LOG2PI
    grad = np.zeros(P)
    for p in np.unique(cnt):
        rows = np.nonzero(cnt == p)[0]
        for a in range(0, rows.shape[0], 4096):
            ri = rows[a:a + 4096]
            S_idx = np.concatenate([nbr[ri, :p].astype(np.int64), ri[:, None]], 1)
            S, dS = _block(kern, X, S_idx)
            yS = y[S_idx]
            N = S[:, :p, :p]
            dN = [D[:, :p, :p] for D in dS]
            nll += 0.5 * float((_l(S, yS) - _l(N, yS[:, :p])).sum())
            grad += 0.5 * (_dl(S, dS, yS) - _dl(N, dN, yS[:, :p])).sum(0)
    return nll, grad


def _dmats(kern, P, Q):
    """Covariance derivative matrices between point sets P and Q, one per parameter."""
    return dcov(kern, P[0][:, None] - Q[0][None, :], P[1][:, None] - Q[1][None, :],
                P[2][:, None] - Q[2][None, :])


def vif_grad(kern, X, y, nbr, Z, jitter=0.0):
    """(NLL, gradient [P]) of the VIF NLL (Sec. "The Vecchia-inducing-point
    full-scale approximation"), from the VIF covariance in dense form.

    The likelihood oracle's VIF is the Gaussian likelihood of
        Sigma_VIF = Sl + B^-1 D B^-T,   Sl = C_nk C_k^-1 C_kn,  C_k = C(Z,Z) + jitter I,
    with B, D the Vecchia factor (neighbor sets nbr) of the residual covariance
        R = C(X,X) + nugget I - Sl.
    Its gradient is the Gaussian formula 1/2 tr(Sigma_VIF^-1 dS) - 1/2 alpha' dS alpha,
    alpha = Sigma_VIF^-1 y, with dS = dSl + d(B^-1 D B^-T) by the chain rule:
        dSl = dC_nk C_k^-1 C_kn + C_nk C_k^-1 dC_kn - C_nk C_k^-1 dC_k C_k^-1 C_kn,
        dR  = dC + dnugget I - dSl,
        dA_i = R_NN^-1 (dR_Ni - dR_NN A_i),   dD_i = dR_ii - 2 A_i . dR_Ni + A_i' dR_NN A_i,
        d(B^-1 D B^-T) = -B^-1 dB V + B^-1 dD B^-T - V dB' B^-T,   V = B^-1 D B^-T,
    where row i of dB holds -dA_i at N(i). Dense n x n algebra: small n only.
    """
    n = X[0].shape[0]
    k = Z[0].shape[0]
    kind = kern["kind"]
    names = PARAMS[kind]
    P = len(names)
    nug = kern["nugget"]
    C = cov_matrix(kern, X, X)
    dC = _dmats(kern, X, X)
    if k > 0:
        Cnk = cov_matrix(kern, X, Z)
        Ck = cov_matrix(kern, Z, Z) + jitter * np.eye(k)
        Cki = np.linalg.inv(Ck)
        dCnk = _dmats(kern, X, Z)
        dCk = _dmats(kern, Z, Z)
        T = Cnk @ Cki                                        # C_nk C_k^-1
        Sl = T @ Cnk.T
        dSl = [dCnk[p] @ T.T + T @ dCnk[p].T - T @ dCk[p] @ T.T for p in range(P)]
    else:
        Sl = np.zeros((n, n))
        dSl = [np.zeros((n, n)) for _ in range(P)]
    R = C + nug * np.eye(n) - Sl
    dR = [dC[p] - dSl[p] for p in range(P)]
    dR[names.index("nugget")] = dR[names.index("nugget")] + np.eye(n)
    # Vecchia factor of R and its derivatives, point by point
    B = np.eye(n)
    D = np.empty(n)
    dB = [np.zeros((n, n)) for _ in range(P)]
    dD = np.empty((P, n))
    for i in range(n):
        N = nbr[i][nbr[i] >= 0].astype(np.int64)
        if N.shape[0] == 0:
            D[i] = R[i, i]
            dD[:, i] = [dR[p][i, i] for p in range(P)]
            continue
        RNN = R[np.ix_(N, N)]
        RNi = R[N, i]
        Ai = np.linalg.solve(RNN, RNi)
        B[i, N] = -Ai
        D[i] = R[i, i] - Ai @ RNi
        for p in range(P):
            dNN = dR[p][np.ix_(N, N)]
            dNi = dR[p][N, i]
            dAi = np.linalg.solve(RNN, dNi - dNN @ Ai)
            dB[p][i, N] = -dAi
            dD[p, i] = dR[p][i, i] - 2.0 * Ai @ dNi + Ai @ dNN @ Ai
    Bi = np.linalg.inv(B)
    V = Bi @ np.diag(D) @ Bi.T
    S = Sl + V
    L = np.linalg.cholesky(S)
    al = np.linalg.solve(S, y)
    nll = 0.5 * n * LOG2PI + float(np.log(np.diag(L)).sum()) + 0.5 * float(y @ al)
    Si = np.linalg.inv(S)
    grad = np.empty(P)
    for p in range(P):
        dV = -Bi @ dB[p] @ V + Bi @ np.diag(dD[p]) @ Bi.T - V @ dB[p].T @ Bi.T
        dS = dSl[p] + dV
        grad[p] = 0.5 * np.einsum("ij,ji->", Si, dS) - 0.5 * float(al @ dS @ al)
    return nll, grad
