"""Pins for the oracle's Vecchia and VIF likelihoods (CPU only).

Each check rests on a fact that holds exactly, not on the oracle itself:
* Vecchia with every earlier point as neighbor is the chain rule of the exact
  likelihood (Sec. "Vecchia approximation"), so it equals the dense Cholesky NLL;
* the closed-form Vecchia NLL equals the dense Gaussian NLL of B^-1 D B^-T;
* D_i is the conditional variance, 1 / (G_S^-1)_ii on the conditioning block;
* KL(exact || Vecchia) >= 0 and does not grow as nested neighbor sets grow,
  and its Monte-Carlo estimate from exact-GP samples agrees;
* VIF with no inducing points is Vecchia, with no neighbors is FITC (Sec.
  "Low-rank inducing point approximations"), with all earlier points as
  neighbors is exact for any inducing set, and with the data as inducing set
  is exact;
* the Woodbury/determinant-lemma assembly equals the dense VIF covariance
  U U' + B^-1 D B^-T;
* the NLL is invariant to permuting inducing points and shifts by n log s when
  y, sigma2 and the nugget are scaled by s, s^2, s^2.
"""
import math

import numpy as np
import pytest

import synth
from oracle import dense, likelihood as LK, neighbors as NB


def _prob(kind=1, n_sites=30, n_times=3, k=8, m=6, seed=0):
    d = synth.config_small(seed=seed, n_sites=n_sites, n_times=n_times, k=k, m=m, kind=kind)
    X = (d["sx"], d["sy"], d["t"])
    Z = (d["zx"], d["zy"], d["zt"]) if k else (np.zeros(0),) * 3
    return d, X, Z


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_vecchia_full_conditioning_is_exact(kind):
    d, X, _ = _prob(kind, k=0)
    n = d["n"]
    nb = NB.brute_force(d["kern"], *X, n - 1)
    v = LK.vecchia(d["kern"], X, d["y"], nb)
    ex = dense.exact_nll(d["kern"], X, d["y"])
    assert abs(v["nll"] - ex) <= 1e-10 * abs(ex)


@pytest.mark.parametrize("m", [0, 1, 5, 12])
def test_vecchia_nll_equals_dense_of_its_factor(m):
    d, X, _ = _prob(1, k=0)
    nb = NB.brute_force(d["kern"], *X, m)
    v = LK.vecchia(d["kern"], X, d["y"], nb)
    S = dense.vecchia_cov(v["A"], v["D"], nb)
    assert abs(v["nll"] - dense.gaussian_nll(S, d["y"])) <= 1e-10 * abs(v["nll"])


def test_D_is_conditional_variance():
    d, X, _ = _prob(1, k=0)
    nb = NB.brute_force(d["kern"], *X, 7)
    v = LK.vecchia(d["kern"], X, d["y"], nb)
    S = dense.exact_cov(d["kern"], X)
    for i in range(d["n"]):
        N = [j for j in nb[i] if j >= 0]
        idx = N + [i]
        P = np.linalg.inv(S[np.ix_(idx, idx)])
        assert abs(v["D"][i] - 1.0 / P[-1, -1]) <= 1e-11 * v["D"][i]


def test_kl_nonnegative_and_monotone_and_monte_carlo():
    d, X, _ = _prob(1, n_sites=40, n_times=3, k=0)
    S = dense.exact_cov(d["kern"], X)
    kls = []
    for m in (1, 3, 6, 12, 24):
        nb = NB.brute_force(d["kern"], *X, m)
        v = LK.vecchia(d["kern"], X, d["y"], nb)
        kls.append(dense.kl_gauss(S, v["A"], v["D"], nb))
    assert min(kls) >= -1e-10
    assert all(b <= a + 1e-10 for a, b in zip(kls, kls[1:])), kls
    nb = NB.brute_force(d["kern"], *X, 3)
    L = np.linalg.cholesky(S)
    rng = np.random.default_rng(11)
    diffs = []
    for _ in range(300):
        y = L @ rng.standard_normal(d["n"])
        diffs.append(LK.vecchia(d["kern"], X, y, nb)["nll"] - dense.gaussian_nll(S, y))
    diffs = np.array(diffs)
    se = diffs.std(ddof=1) / math.sqrt(diffs.shape[0])
    assert abs(diffs.mean() - kls[1]) < 5 * se + 1e-9


@pytest.mark.parametrize("kind", [1, 3])
def test_vif_without_inducing_points_is_vecchia(kind):
    d, X, _ = _prob(kind, k=0)
    nb = NB.brute_force(d["kern"], *X, 6)
    a = LK.vif(d["kern"], X, d["y"], nb, (np.zeros(0),) * 3)
    b = LK.vecchia(d["kern"], X, d["y"], nb)
    assert a["nll"] == b["nll"]


@pytest.mark.parametrize("kind", [1, 2])
def test_vif_without_neighbors_is_fitc(kind):
    d, X, Z = _prob(kind, k=10)
    nb = np.full((d["n"], 0), -1, dtype=np.int32)
    a = LK.vif(d["kern"], X, d["y"], nb, Z)
    b = dense.fitc_nll(d["kern"], X, d["y"], Z)
    assert abs(a["nll"] - b) <= 1e-10 * abs(b)


def test_vif_full_conditioning_is_exact():
    d, X, Z = _prob(1, k=10)
    n = d["n"]
    nb = NB.brute_force(d["kern"], *X, n - 1)
    a = LK.vif(d["kern"], X, d["y"], nb, Z)
    b = dense.exact_nll(d["kern"], X, d["y"])
    assert abs(a["nll"] - b) <= 1e-9 * abs(b)


def test_vif_inducing_at_data_is_exact():
    d, X, _ = _prob(1, n_sites=12, n_times=2, k=0)
    nb = NB.brute_force(d["kern"], *X, 3)
    a = LK.vif(d["kern"], X, d["y"], nb, X)
    b = dense.exact_nll(d["kern"], X, d["y"])
    assert abs(a["nll"] - b) <= 1e-7 * abs(b)
    assert np.allclose(a["D"], d["kern"]["nugget"], rtol=1e-6)


@pytest.mark.parametrize("m", [1, 4, 9])
def test_vif_woodbury_equals_dense(m):
    d, X, Z = _prob(1, k=9)
    nb = NB.brute_force(d["kern"], *X, m)
    a = LK.vif(d["kern"], X, d["y"], nb, Z)
    b = dense.vif_dense_nll(d["kern"], X, d["y"], a["A"], a["D"], nb, Z)
    assert abs(a["nll"] - b) <= 1e-10 * abs(b)


def test_vif_inducing_permutation_invariance():
    d, X, Z = _prob(1, k=9)
    nb = NB.brute_force(d["kern"], *X, 5)
    a = LK.vif(d["kern"], X, d["y"], nb, Z)
    p = np.random.default_rng(2).permutation(Z[0].shape[0])
    b = LK.vif(d["kern"], X, d["y"], nb, tuple(z[p] for z in Z))
    assert abs(a["nll"] - b["nll"]) <= 1e-11 * abs(a["nll"])


def test_vif_scaling():
    d, X, Z = _prob(1, k=9)
    nb = NB.brute_force(d["kern"], *X, 5)
    a = LK.vif(d["kern"], X, d["y"], nb, Z)
    s = 3.0
    kern = dict(d["kern"], sigma2=d["kern"]["sigma2"] * s * s, nugget=d["kern"]["nugget"] * s * s)
    b = LK.vif(kern, X, d["y"] * s, nb, Z)
    assert abs(b["nll"] - (a["nll"] + d["n"] * math.log(s))) <= 1e-10 * abs(b["nll"])


def test_dropped_term_would_be_caught():
    """A plausible slip (forgetting the nugget on the conditioning block) breaks exactness."""
    d, X, _ = _prob(1, k=0)
    nb = NB.brute_force(d["kern"], *X, d["n"] - 1)
    kern0 = dict(d["kern"], nugget=0.0)
    v = LK.vecchia(kern0, X, d["y"], nb)
    ex = dense.exact_nll(d["kern"], X, d["y"])
    assert abs(v["nll"] - ex) > 1e-3
