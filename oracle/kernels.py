"""Covariance kernels in FP64 (oracle; test infrastructure only).

Three kernel kinds, selected by kern["kind"]:

1  GNEITING: the non-separable Gneiting-class kernel written with a stretched
   exponential spatial part,
       psi = a |dt|^(2 alpha) + 1,
       C   = sigma2 * psi^(-tau) * exp(-c * (|ds|^2)^gamma / psi^(beta*gamma)).
   It coincides with Eq. (Gneiting) of the paper for Matern smoothness 1/2
   (paper gamma = 2*beta*gamma, delta = tau - paper gamma, d = 2).

2  GNEITING_MATERN: Eq. (Gneiting) with d = 2 and nu in {1/2, 3/2, 5/2}:
       x = c |ds| / psi^(gamma/2),
       C = sigma2 * psi^-(delta + gamma) * g_nu(x),
   where g_nu is the normalised Matern correlation 2^(1-nu)/Gamma(nu) x^nu K_nu(x).
   The closed forms g_1/2 = e^-x, g_3/2 = (1+x) e^-x, g_5/2 = (1+x+x^2/3) e^-x
   are the elementary expressions the paper's GPU implementation relies on
   (Sec. "GPU acceleration").

3  MATERN_ANISO: Matern on an anisotropic space-time distance,
       d = sqrt(|ds|^2 / range_s^2 + dt^2 / range_t^2),  C = sigma2 * g_nu(d).

All functions return the latent covariance (no nugget).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

GNEITING = 1
GNEITING_MATERN = 2
MATERN_ANISO = 3


def matern_closed(nu, x):
    """Normalised Matern correlation for half-integer nu, elementary closed form."""
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(-x)
    if nu == 0.5:
        return e
    if nu == 1.5:
        return (1.0 + x) * e
    if nu == 2.5:
        return (1.0 + x + x * x / 3.0) * e
    raise ValueError("closed form only for nu in {0.5, 1.5, 2.5}")


def matern_bessel(nu, x):
    """Normalised Matern correlation 2^(1-nu)/Gamma(nu) x^nu K_nu(x), any nu > 0."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    pos = x > 0
    xp = x[pos]
    out[pos] = (2.0 ** (1.0 - nu) / special.gamma(nu)) * xp ** nu * special.kv(nu, xp)
    return out


def _psi(kern, dt):
    return kern["a"] * np.abs(dt) ** (2.0 * kern["alpha"]) + 1.0


def cov(kern, dx, dy, dt, bessel=False):
    """Latent covariance for coordinate differences (dx, dy, dt); broadcasting."""
    dx = np.asarray(dx, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    dt = np.asarray(dt, dtype=np.float64)
    kind = kern["kind"]
    h2 = dx * dx + dy * dy
    if kind == GNEITING:
        psi = _psi(kern, dt)
        g = h2 ** kern["gamma"]
        return kern["sigma2"] * psi ** (-kern["tau"]) * np.exp(
            -kern["c"] * g * psi ** (-kern["beta"] * kern["gamma"]))
    if kind == GNEITING_MATERN:
        psi = _psi(kern, dt)
        gam = kern["gamma"]
        x = kern["c"] * np.sqrt(h2) / psi ** (gam / 2.0)
        g = matern_bessel(kern["nu"], x) if bessel else matern_closed(kern["nu"], x)
        return kern["sigma2"] * psi ** (-(kern["delta"] + gam)) * g
    if kind == MATERN_ANISO:
        rs, rt = kern["range_s"], kern["range_t"]
        d = np.sqrt(h2 / (rs * rs) + dt * dt / (rt * rt))
        g = matern_bessel(kern["nu"], d) if bessel else matern_closed(kern["nu"], d)
        return kern["sigma2"] * g
    raise ValueError(f"unknown kernel kind {kind}")


def cov_matrix(kern, P, Q):
    """Dense latent covariance between point sets P=(sx,sy,t) and Q=(sx,sy,t)."""
    return cov(kern, P[0][:, None] - Q[0][None, :], P[1][:, None] - Q[1][None, :],
               P[2][:, None] - Q[2][None, :])


def correlation(kern, dx, dy, dt, bessel=False):
    """rho = C / sqrt(C_ii C_jj); the kernels are stationary, so C_ii = sigma2."""
    return cov(kern, dx, dy, dt, bessel=bessel) / kern["sigma2"]


def effective_ranges(kern, level=0.05, bessel=False):
    """(time range, space range): the lag / distance at which correlation falls to `level`.

    Time range at zero spatial distance, space range at zero time lag, as used
    in the captions of the paper's parameter tables.
    """
    from scipy.optimize import brentq

    def ft(dt):
        return float(correlation(kern, 0.0, 0.0, dt, bessel)) - level

    def fs(h):
        return float(correlation(kern, h, 0.0, 0.0, bessel)) - level

    def bracket(f, x0):
        hi = x0
        for _ in range(400):
            if f(hi) < 0:
                return hi
            hi *= 2.0
        return math.inf

    hi_t = bracket(ft, 1.0)
    tr = brentq(ft, 0.0, hi_t, xtol=1e-12, rtol=1e-14) if math.isfinite(hi_t) else math.inf
    hi_s = bracket(fs, 1e-12 if kern.get("c", 1.0) > 1e6 else 1e-3)
    sr = brentq(fs, 0.0, hi_s, xtol=1e-14, rtol=1e-14)
    return tr, sr
