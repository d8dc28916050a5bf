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
    with psi_l = a * l^(2 alpha) + 1 at the time lag l = t_i - t_j >= 0.
    The key equals log rho (or a monotone function of it at fixed lag), so
    ranking by key ranks by |rho| for these positive kernels.

Times t_i are real (Sec. "Spatio-temporal Gaussian process model"). The two
lag-only factors of the key depend on the pair only through l; they come from
the C math library once per distinct lag -- a table over l = 0, 1, ... when
every time is an integer, otherwise per distinct value of t_i - t_j (the FP64
difference), with the same operations.
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


def lag_factors(kern, lag):
    """Lag-only factors (f1, f2) of the key at time lag `lag` >= 0, from the C
    math library (Python's math module)."""
    kind = kern["kind"]
    if kind == MATERN_ANISO:
        ir_t = 1.0 / kern["range_t"]
        w = float(lag) * ir_t
        return w * w, 0.0
    psi = kern["a"] * math.pow(float(lag), 2.0 * kern["alpha"]) + 1.0
    if kind == GNEITING:
        return kern["tau"] * math.log(psi), kern["c"] * math.pow(psi, -(kern["beta"] * kern["gamma"]))
    if kind == GNEITING_MATERN:
        return ((kern["delta"] + kern["gamma"]) * math.log(psi),
                kern["c"] * math.pow(psi, -(kern["gamma"] / 2.0)))
    raise ValueError(kind)


def lag_tables(kern, max_lag):
    """Per-lag factors (tab1, tab2) for the integer lags l = 0..max_lag."""
    tab1 = np.zeros(max_lag + 1)
    tab2 = np.zeros(max_lag + 1)
    for lag in range(max_lag + 1):
        tab1[lag], tab2[lag] = lag_factors(kern, lag)
    return tab1, tab2


def integer_times(t):
    return bool(np.all(t == np.round(t)))


def keys(kern, tabs, sx, sy, t, i, js):
    """Ranking keys of candidates js for query i (larger = more correlated).

    tabs = (tab1, tab2) indexed by integer lag, or None: factors per distinct
    lag value (real times)."""
    dx = sx[js] - sx[i]
    dy = sy[js] - sy[i]
    tau = t[i] - t[js]
    if tabs is None:
        lags, inv = np.unique(tau, return_inverse=True)
        f = np.array([lag_factors(kern, v) for v in lags], dtype=np.float64).reshape(-1, 2)
        f1, f2 = f[inv.reshape(-1), 0], f[inv.reshape(-1), 1]
    else:
        lag = tau.astype(np.int64)
        f1, f2 = tabs[0][lag], tabs[1][lag]
    kind = kern["kind"]
    if kind == MATERN_ANISO:
        ir_s = 1.0 / kern["range_s"]
        u = dx * ir_s
        v = dy * ir_s
        return -(f1 + (u * u + v * v))
    h2 = dx * dx + dy * dy
    if kind == GNEITING:
        g = np.sqrt(h2) if kern["gamma"] == 0.5 else np.power(h2, kern["gamma"])
        return -(f1 + g * f2)
    x = np.sqrt(h2) * f2
    nu = kern["nu"]
    if nu == 0.5:
        s = x
    elif nu == 1.5:
        s = np.maximum(x - np.log1p(x), 0.0)
    elif nu == 2.5:
        s = np.maximum(x - np.log1p(x + x * x / 3.0), 0.0)
    else:
        raise ValueError("nu must be 0.5, 1.5 or 2.5")
    return -(f1 + s)


def _check_times(t, integer=False):
    if not np.all(np.isfinite(t)):
        raise ValueError("times must be finite")
    if np.any(np.diff(t) < 0):
        raise ValueError("times must be nondecreasing in index")
    if integer and not integer_times(t):
        raise ValueError("the lag-pruned search takes integer-valued times")


def _rank(keys_, js, m):
    order = np.lexsort((js, -keys_))
    return js[order[:m]], keys_[order[:m]]


def brute_force(kern, sx, sy, t, m, rows=None, general=False):
    """Rank all j < i for each query row; returns int32 [len(rows), m] with -1 padding.

    general=True takes the per-distinct-lag factors even for integer times."""
    _check_times(t)
    n = sx.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    tabs = None
    if n and not general and integer_times(t):
        tabs = lag_tables(kern, int(t[-1] - t[0]))
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
    Integer times only (slabs are the integer time points).
    """
    _check_times(t, integer=True)
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
