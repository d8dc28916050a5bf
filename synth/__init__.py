"""Seeded synthetic inputs for the space-time GP likelihood path.

This module only produces inputs: coordinates in time-stratified random
order, inducing points by kMeans++ on scaled coordinates, and a smooth random
response field. It contains none of the likelihood arithmetic (no covariance
kernel, no Vecchia factor, no low-rank algebra), so that both the FP64 oracle
and the GPU path can consume the same inputs without sharing any code.

Workload shapes follow the paper:
  * simulation geometry: sites uniform on [0,1]^2 observed at equally spaced
    integer times (Sec. "Simulated experiments");
  * station network: a few thousand irregular stations observed daily over a
    year with missing values (Sec. "Data" and the application sections);
  * ordering: sorted by time, locations randomly permuted within each time
    point (Sec. "Correlation-based Vecchia neighbor selection", ordering
    paragraph).

The response is a random-Fourier-feature field plus white noise. It stands in
for a GP sample (the paper's NOAA residuals are not available); the likelihood
value depends on y but parity between oracle and GPU does not.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "time_stratified_order",
    "grid_sites_times",
    "gmm_stations",
    "station_days",
    "kmeanspp",
    "rff_field",
    "config_small",
    "config_cfg1",
    "config_cfg2",
    "config_cfg3",
    "perturb_hyper",
]


def time_stratified_order(sx, sy, t, rng):
    """Sort by time; within each time point apply a seeded random permutation."""
    u = rng.random(t.shape[0])
    order = np.lexsort((u, t))
    return sx[order].copy(), sy[order].copy(), t[order].copy()


def grid_sites_times(n_sites, n_times, rng):
    """Sites uniform on [0,1]^2, each observed at integer times 0..n_times-1."""
    sites = rng.random((n_sites, 2))
    sx = np.tile(sites[:, 0], n_times)
    sy = np.tile(sites[:, 1], n_times)
    t = np.repeat(np.arange(n_times, dtype=np.float64), n_sites)
    return sx, sy, t


def gmm_stations(n_stations, rng, n_comp=40, lon=(-125.0, -67.0), lat=(25.0, 49.0),
                 sd=(0.5, 3.0)):
    """Station lon/lat from a Gaussian mixture, draws outside the box rejected."""
    mu = np.stack([rng.uniform(lon[0], lon[1], n_comp), rng.uniform(lat[0], lat[1], n_comp)], 1)
    sds = rng.uniform(sd[0], sd[1], n_comp)
    w = rng.dirichlet(np.ones(n_comp))
    out = np.empty((0, 2))
    while out.shape[0] < n_stations:
        need = n_stations - out.shape[0]
        comp = rng.choice(n_comp, size=2 * need + 16, p=w)
        pts = mu[comp] + sds[comp, None] * rng.standard_normal((comp.shape[0], 2))
        ok = (pts[:, 0] >= lon[0]) & (pts[:, 0] <= lon[1]) & (pts[:, 1] >= lat[0]) & (pts[:, 1] <= lat[1])
        out = np.concatenate([out, pts[ok]], 0)
    return out[:n_stations]


def project_km(lonlat, lon0=-96.0, lat0=37.0, radius=6371.0):
    """Equirectangular projection to km around (lon0, lat0)."""
    k = math.pi / 180.0
    x = radius * (lonlat[:, 0] - lon0) * k * math.cos(lat0 * k)
    y = radius * (lonlat[:, 1] - lat0) * k
    return x, y


def station_days(n_stations, n_days, missing, rng):
    """Stations (km) observed daily; each (station, day) missing with prob `missing`."""
    xy = project_km(gmm_stations(n_stations, rng))
    sx = np.tile(xy[0], n_days)
    sy = np.tile(xy[1], n_days)
    t = np.repeat(np.arange(n_days, dtype=np.float64), n_stations)
    keep = rng.random(sx.shape[0]) >= missing
    return sx[keep], sy[keep], t[keep]


def kmeanspp(X, k, rng, lloyd_iters=10, lloyd_sample=200_000, seed_sample=100_000, chunk=65536):
    """kMeans++ D^2 seeding on a random subsample, then Lloyd iterations on a subsample.

    X is (n, d) in already scaled coordinates. Returns (k, d) centers.
    """
    if X.shape[0] > seed_sample:
        Xs = X[rng.choice(X.shape[0], seed_sample, replace=False)]
    else:
        Xs = X
    n = Xs.shape[0]
    if k <= 0:
        return np.zeros((0, X.shape[1]))
    centers = np.empty((k, X.shape[1]))
    centers[0] = Xs[rng.integers(n)]
    d2 = ((Xs - centers[0]) ** 2).sum(1)
    for c in range(1, k):
        tot = d2.sum()
        if tot <= 0:
            centers[c] = Xs[rng.integers(n)]
        else:
            r = rng.random() * tot
            idx = int(np.searchsorted(np.cumsum(d2), r, side="right"))
            centers[c] = Xs[min(idx, n - 1)]
        d2 = np.minimum(d2, ((Xs - centers[c]) ** 2).sum(1))
    if lloyd_iters > 0:
        S = X if X.shape[0] <= lloyd_sample else X[rng.choice(X.shape[0], lloyd_sample, replace=False)]
        for _ in range(lloyd_iters):
            lab = np.empty(S.shape[0], dtype=np.int64)
            cn = (centers ** 2).sum(1)
            for a in range(0, S.shape[0], chunk):
                B = S[a:a + chunk]
                lab[a:a + chunk] = np.argmin(cn[None, :] - 2.0 * B @ centers.T, axis=1)
            cnt = np.bincount(lab, minlength=k)
            new = np.zeros_like(centers)
            for j in range(X.shape[1]):
                new[:, j] = np.bincount(lab, weights=S[:, j], minlength=k)
            nz = cnt > 0
            centers[nz] = new[nz] / cnt[nz, None]
    return centers


def inducing_points(sx, sy, t, k, rho_s, rho_t, rng, **kw):
    """kMeans++ on (s/rho_s, t/rho_t); centers mapped back to (sx, sy, t)."""
    X = np.stack([sx / rho_s, sy / rho_s, t / rho_t], 1)
    C = kmeanspp(X, k, rng, **kw)
    return C[:, 0] * rho_s, C[:, 1] * rho_s, C[:, 2] * rho_t


def rff_field(sx, sy, t, rng, ls_s, ls_t, var=1.0, noise=0.1, n_feat=256, chunk=1 << 18):
    """Smooth random field by random Fourier features plus white noise."""
    ws = rng.standard_normal((n_feat, 2)) / ls_s
    wt = rng.standard_normal(n_feat) / ls_t
    ph = rng.uniform(0.0, 2.0 * math.pi, n_feat)
    amp = math.sqrt(2.0 * var / n_feat)
    y = np.empty(sx.shape[0])
    for a in range(0, sx.shape[0], chunk):
        arg = (sx[a:a + chunk, None] * ws[None, :, 0] + sy[a:a + chunk, None] * ws[None, :, 1]
               + t[a:a + chunk, None] * wt[None, :] + ph[None, :])
        y[a:a + chunk] = amp * np.cos(arg).sum(1)
    y += math.sqrt(noise) * rng.standard_normal(sx.shape[0])
    return y


def _pack(sx, sy, t, y, kern, m, ind=None, name=""):
    d = {"name": name, "sx": sx, "sy": sy, "t": t, "y": y, "kern": kern, "m": m, "n": int(sx.shape[0])}
    if ind is not None:
        d["zx"], d["zy"], d["zt"] = ind
        d["k"] = int(ind[0].shape[0])
    else:
        d["k"] = 0
    return d


def kern_matern_aniso(range_s=0.2, range_t=3.0, sigma2=1.0, nugget=0.05, nu=1.5):
    return {"kind": 3, "sigma2": sigma2, "nugget": nugget, "range_s": range_s, "range_t": range_t,
            "nu": nu}


def kern_gneiting(sigma2=1.0, a=0.5, c=20.0, alpha=0.75, beta=0.5, gamma=0.5, tau=1.0, nugget=0.1):
    return {"kind": 1, "sigma2": sigma2, "a": a, "c": c, "alpha": alpha, "beta": beta,
            "gamma": gamma, "tau": tau, "nugget": nugget}


def kern_gneiting_matern(sigma2=1.0, a=0.5, c=20.0, alpha=0.4, gamma=0.4, delta=0.2, nu=1.5,
                         nugget=0.01):
    return {"kind": 2, "sigma2": sigma2, "a": a, "c": c, "alpha": alpha, "gamma": gamma,
            "delta": delta, "nu": nu, "nugget": nugget}


def config_cfg1(seed=0):
    """200 sites x 10 integer times (n=2000), m=10, anisotropic Matern-3/2."""
    rng = np.random.default_rng(seed)
    sx, sy, t = grid_sites_times(200, 10, rng)
    sx, sy, t = time_stratified_order(sx, sy, t, rng)
    kern = kern_matern_aniso()
    y = rff_field(sx, sy, t, rng, ls_s=0.2, ls_t=3.0, noise=kern["nugget"])
    return _pack(sx, sy, t, y, kern, 10, name="cfg1 plain Vecchia n=2000 m=10")


def config_cfg2(seed=0, n_sites=5000, n_times=20, k=500, m=30):
    """5000 sites x 20 days (n=100k), m=30, k=500 kMeans++ inducing points, Gneiting."""
    rng = np.random.default_rng(seed)
    sx, sy, t = grid_sites_times(n_sites, n_times, rng)
    sx, sy, t = time_stratified_order(sx, sy, t, rng)
    kern = kern_gneiting()
    ind = inducing_points(sx, sy, t, k, 0.1498, 11.30, rng)
    y = rff_field(sx, sy, t, rng, ls_s=0.05, ls_t=4.0, noise=kern["nugget"])
    return _pack(sx, sy, t, y, kern, m, ind,
                 name=f"cfg2 VIF n={sx.shape[0]} m={m} k={k}")


def config_cfg3(seed=0, n_stations=3340, n_days=365, k=1000, m=30, missing=0.1):
    """Continental station network (n~1.1M at 3340 stations), m=30, k=1000, Gneiting.

    c and a reproduce effective ranges of 1408 km and 6.7 days (correlation 0.05)
    under the BJ-form Gneiting kernel with alpha=0.75, beta=gamma=0.5, tau=1.
    """
    rng = np.random.default_rng(seed)
    sx, sy, t = station_days(n_stations, n_days, missing, rng)
    sx, sy, t = time_stratified_order(sx, sy, t, rng)
    kern = kern_gneiting(sigma2=1.0, a=1.0956, c=2.1277e-3, alpha=0.75, beta=0.5, gamma=0.5,
                         tau=1.0, nugget=0.1)
    ind = inducing_points(sx, sy, t, k, 1408.0, 6.7, rng, lloyd_iters=5)
    y = rff_field(sx, sy, t, rng, ls_s=400.0, ls_t=3.0, noise=kern["nugget"])
    return _pack(sx, sy, t, y, kern, m, ind,
                 name=f"cfg3 VIF n={sx.shape[0]} m={m} k={k}")


def config_small(seed=0, n_sites=150, n_times=6, k=40, m=12, kind=1, n_stations=None):
    """Small VIF/Vecchia problem for parity tests (ragged rows, several tiles)."""
    rng = np.random.default_rng(seed)
    if n_stations is None:
        sx, sy, t = grid_sites_times(n_sites, n_times, rng)
        ls_s, rho_s = 0.1, 0.15
    else:
        sx, sy, t = station_days(n_stations, n_times, 0.1, rng)
        ls_s, rho_s = 400.0, 1408.0
    sx, sy, t = time_stratified_order(sx, sy, t, rng)
    if kind == 1:
        kern = kern_gneiting() if n_stations is None else kern_gneiting(a=1.0956, c=2.1277e-3)
    elif kind == 2:
        kern = kern_gneiting_matern()
    else:
        kern = kern_matern_aniso()
    ind = inducing_points(sx, sy, t, k, rho_s, 6.0, rng) if k > 0 else None
    y = rff_field(sx, sy, t, rng, ls_s=ls_s, ls_t=3.0, noise=kern["nugget"])
    return _pack(sx, sy, t, y, kern, m, ind, name=f"small n={sx.shape[0]} m={m} k={k}")


def perturb_hyper(kern, rng):
    """Random hyperparameters around `kern`: +-1 in log for scale parameters,
    +-1 in logit for parameters on (0,1)."""
    out = dict(kern)
    for key in ("sigma2", "a", "c", "nugget", "range_s", "range_t"):
        if key in out:
            out[key] = float(out[key] * math.exp(rng.uniform(-1.0, 1.0)))
    for key in ("alpha", "beta", "gamma"):
        if key in out and 0.0 < out[key] < 1.0:
            lg = math.log(out[key] / (1.0 - out[key])) + rng.uniform(-1.0, 1.0)
            out[key] = float(1.0 / (1.0 + math.exp(-lg)))
    return out


def config_station_days(seed=0, n_stations=3340, n_days=30, m=30, missing=0.1, perturb=False,
                        day0=0):
    """Station network over a few days (days day0 .. day0 + n_days - 1), no inducing
    points and no response: the neighbor-search workload (training data of the
    learned proposal when `perturb` draws its hyperparameters around the
    continental kernel)."""
    rng = np.random.default_rng(seed)
    sx, sy, t = station_days(n_stations, n_days, missing, rng)
    sx, sy, t = time_stratified_order(sx, sy, t, rng)
    t = t + float(day0)
    kern = kern_gneiting(sigma2=1.0, a=1.0956, c=2.1277e-3, alpha=0.75, beta=0.5, gamma=0.5,
                         tau=1.0, nugget=0.1)
    if perturb:
        kern = perturb_hyper(kern, rng)
    return {"sx": sx, "sy": sy, "t": t, "kern": kern, "m": m, "n": int(sx.shape[0]), "k": 0,
            "name": f"stations n={sx.shape[0]} m={m}"}


def config_batch(seed=0, count=64, n_lo=10_000, n_hi=200_000, ms=(10, 20, 30), ks=(200, 500),
                 n_stations=3340, missing=0.1):
    """Independent station-network problems for batched evaluation: n log-uniform
    in [n_lo, n_hi] (a time-ordered prefix of a station network observed daily),
    m and k drawn from `ms` and `ks`, hyperparameters drawn around the
    continental kernel (perturb_hyper), k kMeans++ inducing points, a smooth
    random response."""
    rng = np.random.default_rng(seed)
    base = kern_gneiting(sigma2=1.0, a=1.0956, c=2.1277e-3, alpha=0.75, beta=0.5, gamma=0.5,
                         tau=1.0, nugget=0.1)
    out = []
    for b in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        m = int(rng.choice(ms))
        k = int(rng.choice(ks))
        n_days = max(2, int(math.ceil(n / (n_stations * (1.0 - missing)))) + 1)
        sx, sy, t = station_days(n_stations, n_days, missing, rng)
        sx, sy, t = time_stratified_order(sx, sy, t, rng)
        sx, sy, t = sx[:n], sy[:n], t[:n]
        kern = perturb_hyper(base, rng)
        ind = inducing_points(sx, sy, t, k, 1408.0, 6.7, rng, lloyd_iters=2, seed_sample=20_000,
                              lloyd_sample=50_000)
        y = rff_field(sx, sy, t, rng, ls_s=400.0, ls_t=3.0, noise=kern["nugget"], n_feat=64)
        out.append(_pack(sx, sy, t, y, kern, m, ind, name=f"batch[{b}] n={n} m={m} k={k}"))
    return out
