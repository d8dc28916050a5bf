"""Correlation-based Vecchia neighbor sets (oracle; test infrastructure only).

Definition (Sec. "Correlation-based Vecchia neighbor selection"): point i takes
as neighbors the min(i, m) points j < i that are closest in the correlation
metric d_c = sqrt(1 - |rho_ij|), i.e. of largest |rho_ij| under the latent
kernel (the nugget is not part of Sigma). Neighbors come only from earlier
indices (the index-ordered insertion of Alg. 1 and the "index < i" restriction
of Alg. 2); Alg. 2 is an exact nearest-neighbor search, so the plain definition
-- rank every earlier point -- gives the same sets.

Readings taken where the paper is silent:
  * ties in correlation go to the lower index;
  * rows are ordered by decreasing correlation, then increasing index, and a
    row with fewer than m earlier points is padded with -1;
  * the ranking key is the log-correlation evaluated with a fixed operation
    order in IEEE FP64 (no fused multiply-add), with the per-lag factors taken
    from the C math library, so that an independent implementation can
    reproduce the sets bit for bit:
        GNEITING          key = -(tau*log(psi_l) + g * c*psi_l^(-beta*gamma)),
                          g = sqrt(h2) when gamma == 1/2 else h2^gamma
        GNEITING_MATERN   key = -((delta+gamma)*log(psi_l) + s(x)),
                          x = sqrt(h2) * c*psi_l^(-gamma/2),
                          s(x) = x - log g_nu(x) e^x  (= x for nu = 1/2)
        MATERN_ANISO      key = -((u*u + v*v) + w*w),  u = dx/range_s, ...
                          (minus the squared anisotropic distance; the Matern
                          correlation is decreasing in the distance)
    with psi_l = a * l^(2 alpha) + 1 at integer lag l = t_i - t_j.
    The key equals log rho (or a monotone function of it at fixed lag), so
    ranking by key ranks by |rho| for these positive kernels.
"""
from __future__ import annotations

import math

import numpy as np

from .kernels import GNEITING, GNEITING_MATERN, MATERN_ANISO, correlation


def key_is_exact(kern):
    """True when the key needs only IEEE add, mul and sqrt per pair."""
    k = kern["kind"]
    if k == GNEITING:
        return kern["gamma"] == 0.5
    if k == GNEITING_MATERN:
        return kern["nu"] == 0.5
    return True


def lag_tables(kern, max_lag):
    """Per-lag factors (tab1, tab2) for l = 0..max_lag, from the C math library."""
    kind = kern["kind"]
    tab1 = np.zeros(max_lag + 1)
    tab2 = np.zeros(max_lag + 1)
    if kind == MATERN_ANISO:
        ir_t = 1.0 / kern["range_t"]
        for lag in range(max_lag + 1):
            w = float(lag) * ir_t
            tab1[lag] = w * w
        return tab1, tab2
    a, two_alpha = kern["a"], 2.0 * kern["alpha"]
    for lag in range(max_lag + 1):
        psi = a * math.pow(float(lag), two_alpha) + 1.0
        if kind == GNEITING:
            tab1[lag] = kern["tau"] * math.log(psi)
            tab2[lag] = kern["c"] * math.pow(psi, -(kern["beta"] * kern["gamma"]))
        elif kind == GNEITING_MATERN:
            tab1[lag] = (kern["delta"] + kern["gamma"]) * math.log(psi)
            tab2[lag] = kern["c"] * math.pow(psi, -(kern["gamma"] / 2.0))
        else:
            raise ValueError(kind)
    return tab1, tab2


def keys(kern, tabs, sx, sy, t, i, js):
    """Ranking keys of candidates js for query i (larger = more correlated)."""
    tab1, tab2 = tabs
    dx = sx[js] - sx[i]
    dy = sy[js] - sy[i]
    lag = (t[i] - t[js]).astype(np.int64)
    kind = kern["kind"]
    if kind == MATERN_ANISO:
        ir_s = 1.0 / kern["range_s"]
        u = dx * ir_s
        v = dy * ir_s
        return -(tab1[lag] + (u * u + v * v))
    h2 = dx * dx + dy * dy
    if kind == GNEITING:
        g = np.sqrt(h2) if kern["gamma"] == 0.5 else np.power(h2, kern["gamma"])
        return -(tab1[lag] + g * tab2[lag])
    x = np.sqrt(h2) * tab2[lag]
    nu = kern["nu"]
    if nu == 0.5:
        s = x
    elif nu == 1.5:
        s = np.maximum(x - np.log1p(x), 0.0)
    elif nu == 2.5:
        s = np.maximum(x - np.log1p(x + x * x / 3.0), 0.0)
    else:
        raise ValueError("nu must be 0.5, 1.5 or 2.5")
    return -(tab1[lag] + s)


def _check_times(t):
    if np.any(np.diff(t) < 0):
        raise ValueError("times must be nondecreasing in index")
    if np.any(t != np.round(t)):
        raise ValueError("neighbor search requires integer-valued times")


def _rank(keys_, js, m):
    order = np.lexsort((js, -keys_))
    return js[order[:m]], keys_[order[:m]]


def brute_force(kern, sx, sy, t, m, rows=None):
    """Rank all j < i for each query row; returns int32 [len(rows), m] with -1 padding."""
    _check_times(t)
    n = sx.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    max_lag = int(t[-1] - t[0]) if n else 0
    tabs = lag_tables(kern, max_lag)
    out = np.full((rows.shape[0], m), -1, dtype=np.int32)
    for r, i in enumerate(rows):
        if i == 0 or m == 0:
            continue
        js = np.arange(i)
        sel, _ = _rank(keys(kern, tabs, sx, sy, t, i, js), js, m)
        out[r, :sel.shape[0]] = sel
    return out


def lag_pruned(kern, sx, sy, t, m, rows=None):
    """Same result as brute_force, visiting time slabs in increasing lag and stopping
    once no later slab can beat the current m-th key.

    The key of a pair at lag l is never above -tab1[l] (the spatial term is
    nonnegative and IEEE addition is monotone), so after suffix maximisation the
    bound holds for every larger lag as well. Scanning continues while the bound
    equals the m-th key, since a lower index could still win the tie.
    """
    _check_times(t)
    n = sx.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    out = np.full((rows.shape[0], m), -1, dtype=np.int32)
    if n == 0 or m == 0:
        return out
    t0 = t[0]
    max_lag = int(t[-1] - t0)
    tabs = lag_tables(kern, max_lag)
    bound = -tabs[0]
    bound = np.maximum.accumulate(bound[::-1])[::-1]
    for r, i in enumerate(rows):
        ti = t[i]
        best_j = np.zeros(0, dtype=np.int64)
        best_k = np.zeros(0)
        for lag in range(int(ti - t0) + 1):
            if best_j.shape[0] >= m and bound[lag] < best_k[m - 1]:
                break
            tv = ti - lag
            lo = int(np.searchsorted(t, tv, side="left"))
            hi = i if lag == 0 else int(np.searchsorted(t, tv, side="right"))
            if hi <= lo:
                continue
            js = np.arange(lo, hi)
            kk = keys(kern, tabs, sx, sy, t, i, js)
            best_j, best_k = _rank(np.concatenate([best_k, kk]), np.concatenate([best_j, js]), m)
        out[r, :best_j.shape[0]] = best_j
    return out


def rho_order_mismatches(kern, sx, sy, t, nbr, rows):
    """Rows whose neighbor order under the exp-based FP64 correlation differs from
    the key order (near-ties between the two evaluations)."""
    bad = []
    for r, i in enumerate(rows):
        js = nbr[r][nbr[r] >= 0].astype(np.int64)
        if js.shape[0] < 2:
            continue
        rho = correlation(kern, sx[js] - sx[i], sy[js] - sy[i], t[i] - t[js])
        if np.any(np.diff(rho) > 0):
            bad.append(int(i))
    return bad
