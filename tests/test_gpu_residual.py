"""Residual-correlation neighbors (include/vif_residual.h) against the FP64 oracle.

Bar: the GPU forms each key from an FP64 MFMA Gram and its own covariance
evaluation, so keys agree with the oracle's to rounding (about 1e-15 relative)
and sets can differ only where two candidates' keys are that close. Every row is
checked: either it equals the oracle's row, or it holds min(i, m) distinct
earlier points, in non-increasing oracle-key order up to that rounding, whose
keys match the oracle's top keys to 1e-9 relative; such near-tie rows must stay
rare (under 1 %). A query without residual variance (r(i, i) <= 1e-10 sigma2: a point
that coincides with an inducing point, e.g. the centre of a one-point kMeans
cluster) has a residual correlation of 0/0 with every candidate, its keys are
rounding noise on both sides, and any valid row is accepted for it. At the benchmark size (cfg2: n = 100,000, k = 500) sampled rows
are checked the same way against the oracle run on those rows only.
"""
import numpy as np
import pytest

import synth
from oracle import residual as RS
from tests.gpu_util import dev, lib, log, problem_on_device, torch_cuda

pytestmark = pytest.mark.gpu


def _check_rows(kern, X, Z, got, rows, m, U=None, dv=None):
    want = RS.brute_force(kern, X, Z, m, rows=rows) if rows is not None else RS.brute_force(kern, X, Z, m)
    rows = np.arange(X[0].shape[0]) if rows is None else np.asarray(rows)
    if U is None:
        U, dv = RS.residual_parts(kern, X, Z)
    near = 0
    for r, i in enumerate(rows):
        g, w = got[r], want[r]
        if np.array_equal(g, w):
            continue
        cnt = min(int(i), m)
        gv = g[g >= 0]
        assert gv.shape[0] == cnt and np.all(g[cnt:] == -1), (i, g, w)
        assert np.unique(gv).shape[0] == cnt and np.all(gv < i), (i, g)
        if dv[i] <= 1e-10 * kern["sigma2"]:
            continue  # 0/0: no residual at the query (not counted)
        near += 1
        kg = RS.row_keys(kern, X, U, dv, i, gv)
        kw = RS.row_keys(kern, X, U, dv, i, w[:cnt])
        assert np.allclose(kg, kw, rtol=1e-9, atol=0.0), (i, kg, kw)
        assert np.all(np.diff(kg) <= 1e-9 * np.abs(kg[:-1])), (i, kg)
    return near


CASES = {
    "gneit_k40_m12": dict(seed=41, n_sites=150, n_times=6, k=40, m=12, kind=1),
    "gneitmatern_k30_m8": dict(seed=42, n_sites=120, n_times=5, k=30, m=8, kind=2),
    "stations_k60_m30": dict(seed=43, n_times=5, k=60, m=30, kind=1, n_stations=250),
    "aniso_k70_m20": dict(seed=44, n_sites=100, n_times=7, k=70, m=20, kind=3),
    "gneit_k0_m10": dict(seed=45, n_sites=130, n_times=5, k=0, m=10, kind=1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_residual_neighbors_match_oracle(name):
    torch = torch_cuda()
    vif = lib()
    d = synth.config_small(**CASES[name])
    X = (d["sx"], d["sy"], d["t"])
    Z = (d["zx"], d["zy"], d["zt"]) if d["k"] else None
    Xd, _, Zd = problem_on_device(d)
    got = vif.vif_residual_neighbors(*Xd, d["kern"], d["m"], ind=Zd).cpu().numpy()
    near = _check_rows(d["kern"], X, Z, got, None, d["m"])
    log(f"[residual] {name} n={d['n']} k={d['k']} m={d['m']}: near-tie rows {near}")
    assert near <= 0.01 * d["n"]


def test_point_at_inducing_point_is_not_chosen():
    torch = torch_cuda()
    vif = lib()
    d = synth.config_small(seed=46, n_sites=80, n_times=4, k=12, m=8, kind=1)
    j = 9
    d["zx"][0], d["zy"][0], d["zt"][0] = d["sx"][j], d["sy"][j], d["t"][j]
    Xd, _, Zd = problem_on_device(d)
    got = vif.vif_residual_neighbors(*Xd, d["kern"], d["m"], ind=Zd).cpu().numpy()
    for i in range(j + 10, d["n"]):
        assert j not in got[i]


def test_m_one_and_first_rows():
    torch = torch_cuda()
    vif = lib()
    d = synth.config_small(seed=47, n_sites=70, n_times=3, k=20, m=1, kind=2)
    X = (d["sx"], d["sy"], d["t"])
    Z = (d["zx"], d["zy"], d["zt"])
    Xd, _, Zd = problem_on_device(d)
    for m in (1, 63):
        got = vif.vif_residual_neighbors(*Xd, d["kern"], m, ind=Zd).cpu().numpy()
        assert got[0].tolist() == [-1] * m
        near = _check_rows(d["kern"], X, Z, got, None, m)
        assert near <= 0.01 * d["n"]


def test_benchmark_size_sampled_rows():
    torch = torch_cuda()
    vif = lib()
    d = synth.config_cfg2()
    X = (d["sx"], d["sy"], d["t"])
    Z = (d["zx"], d["zy"], d["zt"])
    Xd, _, Zd = problem_on_device(d)
    got = vif.vif_residual_neighbors(*Xd, d["kern"], d["m"], ind=Zd).cpu().numpy()
    n = d["n"]
    rows = np.unique(np.concatenate([np.arange(5), np.random.default_rng(0).integers(0, n, 40),
                                     np.arange(n - 5, n)]))
    U, dv = RS.residual_parts(d["kern"], X, Z)
    near = _check_rows(d["kern"], X, Z, got[rows], rows, d["m"], U, dv)
    log(f"[residual] cfg2 n={n}: {rows.shape[0]} sampled rows, near-tie rows {near}")
    assert near <= 2
