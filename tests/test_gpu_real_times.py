"""Neighbor search with real-valued times (Sec. "Spatio-temporal Gaussian process
model": t_i is real) against the FP64 oracle's plain definition (brute force over
all earlier points, lag-only factors per distinct lag from the host C math
library).

On the device each pair's lag factors come from the device pow and log, which
can differ from the host library by an ulp, so two candidates whose keys agree
to rounding may swap. The bar: every row either equals the oracle's or holds
min(i, m) distinct earlier points, -1 padded, in non-increasing oracle-key order
up to 1e-12 relative, with the same multiset of keys as the oracle's row to
1e-12 relative; such near-tie rows must be rare (at most 1 %). Cases: measurement
times scattered within days, a mix of integer and fractional times with ties, a
far time origin, and a single common fractional time.
"""
import zlib

import numpy as np
import pytest

import synth
from oracle import neighbors as NB
from tests.gpu_util import lib, log, problem_on_device, torch_cuda

pytestmark = pytest.mark.gpu

KERNELS = {
    "gneiting": synth.kern_gneiting(),
    "gneiting_g04": synth.kern_gneiting(gamma=0.4, beta=0.6),
    "gm_nu05": synth.kern_gneiting_matern(nu=0.5),
    "gm_nu15": synth.kern_gneiting_matern(nu=1.5),
    "gm_nu25": synth.kern_gneiting_matern(nu=2.5),
    "aniso": synth.kern_matern_aniso(),
}


def times(kind, n_sites, rng):
    if kind == "scattered":      # 8 days, each site observed once a day at a random hour
        t = np.repeat(np.arange(8.0), n_sites) + rng.random(8 * n_sites) * 0.99
    elif kind == "mixed":        # integer days and half days, many equal times
        t = np.repeat(np.arange(0.0, 5.0, 0.5), n_sites)[: 8 * n_sites]
    elif kind == "far_origin":   # an origin far from zero
        t = 1000.25 + np.repeat(np.arange(8.0), n_sites) * 0.75 + rng.random(8 * n_sites) * 0.1
    else:                        # one common fractional time
        t = np.full(8 * n_sites, 2.5)
    return t


def check_rows(kern, sx, sy, t, got, m):
    n = sx.shape[0]
    want = NB.brute_force(kern, sx, sy, t, m)
    near = 0
    for i in range(n):
        g, w = got[i], want[i]
        if np.array_equal(g, w):
            continue
        cnt = min(i, m)
        gv = g[:cnt]
        assert np.all(g[cnt:] == -1) and np.all(gv >= 0) and np.all(gv < i), (i, g)
        assert np.unique(gv).shape[0] == cnt, (i, g)
        kg = NB.keys(kern, None, sx, sy, t, i, gv.astype(np.int64))
        kw = NB.keys(kern, None, sx, sy, t, i, w[:cnt].astype(np.int64))
        tol = 1e-12 * np.maximum(np.abs(kw), 1e-300)
        assert np.all(np.abs(np.sort(kg) - np.sort(kw)) <= tol), (i, kg, kw)
        assert np.all(np.diff(kg) <= 1e-12 * np.abs(kg[:-1]) + 1e-300), (i, kg)
        near += 1
    return near


@pytest.mark.parametrize("tkind", ["scattered", "mixed", "far_origin", "single"])
@pytest.mark.parametrize("name", list(KERNELS))
def test_real_times_match_oracle(name, tkind):
    torch = torch_cuda()
    vif = lib()
    kern = KERNELS[name]
    rng = np.random.default_rng(zlib.crc32(f"{name}:{tkind}".encode()))
    n_sites = 140
    sites = rng.random((n_sites, 2))
    sx = np.tile(sites[:, 0], 8)
    sy = np.tile(sites[:, 1], 8)
    t = times(tkind, n_sites, rng)
    sx, sy, t = synth.time_stratified_order(sx, sy, t, rng)
    m = 20
    log(f"[real times] {name} {tkind} n={sx.shape[0]} m={m}")
    d = {"sx": sx, "sy": sy, "t": t, "y": np.zeros_like(sx), "k": 0}
    Xd, _, _ = problem_on_device(d)
    got = vif.vif_neighbors(*Xd, kern, m).cpu().numpy()
    torch.cuda.synchronize()
    near = check_rows(kern, sx, sy, t, got, m)
    log(f"[real times] {name} {tkind}: near-tie rows {near}")
    assert near <= 0.01 * sx.shape[0]


def test_real_times_combined_call_and_nll():
    """The combined search + NLL call on real times gives the same rows as the
    search alone and an NLL within 1e-8 of the oracle's on those rows."""
    torch = torch_cuda()
    vif = lib()
    from oracle import likelihood as LK
    rng = np.random.default_rng(91)
    d = synth.config_small(seed=9, n_sites=120, n_times=6, k=30, m=12, kind=1)
    t = d["t"] + rng.random(d["n"]) * 0.9
    sx, sy, t = synth.time_stratified_order(d["sx"], d["sy"], t, rng)
    d2 = dict(d, sx=sx, sy=sy, t=t)
    Xd, yd, Zd = problem_on_device(d2)
    nb = vif.vif_neighbors(*Xd, d["kern"], d["m"])
    v, nb2 = vif.vif_neighbors_nll(*Xd, yd, d["kern"], d["m"], ind=Zd, prec="fp64")
    assert torch.equal(nb, nb2)
    nbh = nb.cpu().numpy()
    ref = LK.vif(d["kern"], (sx, sy, t), d["y"], nbh, (d["zx"], d["zy"], d["zt"]))["nll"]
    log(f"[real times] combined nll {v:.12g} oracle {ref:.12g}")
    assert abs(v - ref) <= 1e-8 * abs(ref)
