"""Pins for the oracle's Vecchia NLL gradient (CPU only).

* each covariance derivative equals a central finite difference of the oracle's
  covariance (a separately pinned function) in that parameter, for the three
  kernel families (Gneiting-Matern with each closed-form smoothness);
* the gradient equals central finite differences of the oracle's Vecchia NLL
  (pinned against the dense exact likelihood);
* with m = n - 1 the Vecchia likelihood is exact, so the gradient equals the
  dense Gaussian gradient 1/2 tr(S^-1 dS) - 1/2 y'S^-1 dS S^-1 y of the full
  covariance, evaluated here by finite differences of the dense exact NLL;
* the NLL it returns equals the likelihood oracle's.
"""
import numpy as np
import pytest

import synth
from oracle import dense as DN
from oracle import gradient as GR
from oracle import kernels as K
from oracle import likelihood as LK
from oracle import neighbors as NB


KINDS = {"gneiting": 1, "gm_nu05": 2, "gm_nu15": 2, "gm_nu25": 2, "aniso": 3}


def _kern(name):
    if name == "gneiting":
        return synth.kern_gneiting(sigma2=1.3, a=0.7, c=15.0, alpha=0.6, beta=0.4, gamma=0.45,
                                   tau=1.2, nugget=0.08)
    if name.startswith("gm_"):
        nu = {"gm_nu05": 0.5, "gm_nu15": 1.5, "gm_nu25": 2.5}[name]
        return synth.kern_gneiting_matern(sigma2=1.1, a=0.6, c=8.0, alpha=0.45, gamma=0.35,
                                          delta=0.3, nu=nu, nugget=0.06)
    return synth.kern_matern_aniso(range_s=0.25, range_t=2.5, sigma2=0.9, nugget=0.07, nu=1.5)


def _bump(kern, name, h):
    out = dict(kern)
    out[name] = kern[name] + h
    return out


@pytest.mark.parametrize("name", list(KINDS))
def test_covariance_derivatives_match_finite_differences(name):
    kern = _kern(name)
    kind = KINDS[name]
    rng = np.random.default_rng(len(name) + kind)
    dx, dy = rng.normal(scale=0.2, size=200), rng.normal(scale=0.2, size=200)
    dt = rng.integers(-4, 5, size=200).astype(float)
    dx[:5] = dy[:5] = 0.0      # same place
    dt[5:10] = 0.0             # same time
    D = GR.dcov(kern, dx, dy, dt)
    for p, par in enumerate(GR.PARAMS[kind]):
        if par == "nugget":
            assert np.all(D[p] == 0.0)
            continue
        h = 1e-6 * max(abs(kern[par]), 1e-3)
        fd = (K.cov(_bump(kern, par, h), dx, dy, dt) - K.cov(_bump(kern, par, -h), dx, dy, dt)) / (2 * h)
        assert np.allclose(D[p], fd, rtol=1e-5, atol=1e-8), par


def _fd_grad(f, kern, names):
    g = []
    for name in names:
        h = 1e-5 * max(abs(kern[name]), 1e-3)
        g.append((f(_bump(kern, name, h)) - f(_bump(kern, name, -h))) / (2 * h))
    return np.array(g)


@pytest.mark.parametrize("name", list(KINDS))
def test_gradient_matches_finite_differences_of_the_nll(name):
    kind = KINDS[name]
    d = synth.config_small(seed=10 + kind, n_sites=40, n_times=4, k=0, m=6, kind=kind)
    kern = _kern(name)
    X = (d["sx"], d["sy"], d["t"])
    nbr = NB.brute_force(kern, *X, 6)
    nll, g = GR.vecchia_grad(kern, X, d["y"], nbr)
    assert abs(nll - LK.vecchia(kern, X, d["y"], nbr)["nll"]) < 1e-9 * abs(nll)
    fd = _fd_grad(lambda k: LK.vecchia(k, X, d["y"], nbr)["nll"], kern, GR.PARAMS[kind])
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())


@pytest.mark.parametrize("name", list(KINDS))
def test_full_conditioning_gives_the_exact_gradient(name):
    kind = KINDS[name]
    d = synth.config_small(seed=20 + kind, n_sites=15, n_times=3, k=0, m=6, kind=kind)
    kern = _kern(name)
    X = (d["sx"], d["sy"], d["t"])
    n = d["n"]
    nbr = NB.brute_force(kern, *X, n - 1)
    _, g = GR.vecchia_grad(kern, X, d["y"], nbr)
    fd = _fd_grad(lambda k: DN.exact_nll(k, X, d["y"]), kern, GR.PARAMS[kind])
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())


@pytest.mark.parametrize("name", list(KINDS))
def test_vif_gradient_matches_finite_differences_of_the_vif_nll(name):
    """The VIF gradient (dense chain rule) against central differences of the
    pinned VIF likelihood oracle (Woodbury form), inducing points and
    neighbor sets held fixed; its NLL equals the likelihood oracle's."""
    kind = KINDS[name]
    d = synth.config_small(seed=30 + kind, n_sites=30, n_times=4, k=12, m=5, kind=kind)
    kern = _kern(name)
    X = (d["sx"], d["sy"], d["t"])
    Z = (d["zx"], d["zy"], d["zt"])
    nbr = NB.brute_force(kern, *X, 5)
    nll, g = GR.vif_grad(kern, X, d["y"], nbr, Z)
    ref = LK.vif(kern, X, d["y"], nbr, Z)["nll"]
    assert abs(nll - ref) < 1e-10 * abs(ref)
    fd = _fd_grad(lambda k: LK.vif(k, X, d["y"], nbr, Z)["nll"], kern, GR.PARAMS[kind])
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())


def test_vif_gradient_without_inducing_points_is_the_vecchia_gradient():
    d = synth.config_small(seed=41, n_sites=30, n_times=3, k=0, m=6, kind=1)
    kern = _kern("gneiting")
    X = (d["sx"], d["sy"], d["t"])
    nbr = NB.brute_force(kern, *X, 6)
    empty = (np.zeros(0), np.zeros(0), np.zeros(0))
    nll, g = GR.vif_grad(kern, X, d["y"], nbr, empty)
    nll_v, g_v = GR.vecchia_grad(kern, X, d["y"], nbr)
    assert abs(nll - nll_v) < 1e-10 * abs(nll_v)
    assert np.allclose(g, g_v, rtol=1e-9, atol=1e-10 * np.abs(g_v).max())


@pytest.mark.parametrize("name", ["gneiting", "gm_nu25", "aniso"])
def test_vif_gradient_with_full_conditioning_is_the_exact_gradient(name):
    """m = n - 1: VIF is exact for any inducing points, so its gradient is the
    gradient of the dense exact NLL (finite differences)."""
    kind = KINDS[name]
    d = synth.config_small(seed=50 + kind, n_sites=12, n_times=3, k=7, m=4, kind=kind)
    kern = _kern(name)
    X = (d["sx"], d["sy"], d["t"])
    Z = (d["zx"], d["zy"], d["zt"])
    n = d["n"]
    nbr = NB.brute_force(kern, *X, n - 1)
    _, g = GR.vif_grad(kern, X, d["y"], nbr, Z)
    fd = _fd_grad(lambda k: DN.exact_nll(k, X, d["y"]), kern, GR.PARAMS[kind])
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())
