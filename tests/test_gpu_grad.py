"""Gradient of the Vecchia NLL (include/vif_grad.h) against the FP64 oracle.

Cases cover the three kernel families (Gneiting-Matern at nu = 1/2, 3/2, 5/2).
Bars (all arithmetic is FP64 on both sides; only the order of operations
differs): NLL within 1e-10 relative of the oracle and of vif_nll; every
gradient entry within 1e-8 of the largest entry's magnitude. Repeated calls
are bit-identical (fixed-order sums).
"""
import numpy as np
import pytest

import synth
from oracle import gradient as GR
from oracle import neighbors as NB
from tests.gpu_util import dev, lib, log, problem_on_device, rel, torch_cuda

pytestmark = pytest.mark.gpu


def _kern(kind, nu=1.5):
    if kind == 1:
        return synth.kern_gneiting(sigma2=1.3, a=0.7, c=15.0, alpha=0.6, beta=0.4, gamma=0.45,
                                   tau=1.2, nugget=0.08)
    if kind == 2:
        return synth.kern_gneiting_matern(sigma2=1.1, a=0.6, c=8.0, alpha=0.45, gamma=0.35,
                                          delta=0.3, nu=nu, nugget=0.06)
    return synth.kern_matern_aniso(range_s=0.25, range_t=2.5, sigma2=0.9, nugget=0.07, nu=1.5)


CASES = {
    "gneit_m6": (1, dict(seed=51, n_sites=150, n_times=5, k=0, m=6, kind=1)),
    "gneit_m30": (1, dict(seed=52, n_sites=200, n_times=5, k=0, m=30, kind=1)),
    "gneit_m40": (1, dict(seed=53, n_sites=120, n_times=6, k=0, m=40, kind=1)),
    "gm_nu05_m12": ((2, 0.5), dict(seed=57, n_sites=150, n_times=5, k=0, m=12, kind=2)),
    "gm_nu15_m30": ((2, 1.5), dict(seed=58, n_sites=160, n_times=6, k=0, m=30, kind=2)),
    "gm_nu25_m50": ((2, 2.5), dict(seed=59, n_sites=110, n_times=6, k=0, m=50, kind=2)),
    "aniso_m10": (3, dict(seed=54, n_sites=200, n_times=6, k=0, m=10, kind=3)),
    "aniso_m63": (3, dict(seed=55, n_sites=100, n_times=7, k=0, m=63, kind=3)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_gradient_matches_oracle(name):
    torch = torch_cuda()
    vif = lib()
    kind, cfg = CASES[name]
    d = synth.config_small(**cfg)
    kern = _kern(*kind) if isinstance(kind, tuple) else _kern(kind)
    X = (d["sx"], d["sy"], d["t"])
    m = cfg["m"]
    nbr = NB.brute_force(kern, *X, m)
    Xd, yd, _ = problem_on_device(d)
    nb = dev(nbr, torch.int32)
    nll, g = vif.vif_nll_grad(*Xd, yd, kern, m, nb)
    want_nll, want_g = GR.vecchia_grad(kern, X, d["y"], nbr)
    err = np.abs(np.array(g) - want_g).max() / np.abs(want_g).max()
    log(f"[grad] {name} n={d['n']} m={m}: nll rel {rel(nll, want_nll):.2e}, grad err {err:.2e}")
    assert rel(nll, want_nll) <= 1e-10
    assert rel(nll, vif.vif_nll(*Xd, yd, kern, m, nb, prec="fp64")) <= 1e-10
    assert err <= 1e-8
    nll2, g2 = vif.vif_nll_grad(*Xd, yd, kern, m, nb)
    assert nll2 == nll and g2 == g


def test_bad_neighbor_row_is_rejected():
    torch = torch_cuda()
    vif = lib()
    d = synth.config_small(seed=56, n_sites=60, n_times=4, k=0, m=8, kind=1)
    kern = _kern(1)
    X = (d["sx"], d["sy"], d["t"])
    nbr = NB.brute_force(kern, *X, 8)
    nbr[20, 2] = 25  # not an earlier point
    Xd, yd, _ = problem_on_device(d)
    with pytest.raises(vif.VifError):
        vif.vif_nll_grad(*Xd, yd, kern, 8, dev(nbr, torch.int32))


def test_gradient_at_workload_size():
    """Station network over 30 days (n ~ 90k), m = 30, Gneiting kernel of the
    continental workload: the whole gradient against the oracle."""
    torch = torch_cuda()
    vif = lib()
    d = synth.config_station_days(seed=3, n_days=30, m=30)
    rng = np.random.default_rng(3)
    d["y"] = rng.normal(size=d["n"])
    kern = d["kern"]
    X = (d["sx"], d["sy"], d["t"])
    Xd = tuple(dev(d[k], torch.float64) for k in ("sx", "sy", "t"))
    yd = dev(d["y"], torch.float64)
    nb = vif.vif_neighbors(*Xd, kern, 30)
    nll, g = vif.vif_nll_grad(*Xd, yd, kern, 30, nb)
    want_nll, want_g = GR.vecchia_grad(kern, X, d["y"], nb.cpu().numpy())
    err = np.abs(np.array(g) - want_g).max() / np.abs(want_g).max()
    log(f"[grad] stations n={d['n']}: nll rel {rel(nll, want_nll):.2e}, grad err {err:.2e}")
    assert rel(nll, want_nll) <= 1e-10
    assert err <= 1e-8
