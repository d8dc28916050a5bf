"""GPU gradient of the VIF NLL (vif_nll_grad_vif, through the C ABI) against
the FP64 oracle's dense-form gradient (oracle.gradient.vif_grad, pinned by
central differences of the VIF likelihood oracle).

Bars: NLL within 1e-10 relative of the oracle's; every gradient entry within
1e-8 of the largest entry's magnitude. Cases: the three kernel families,
Gneiting-Matern at nu = 1/2, 3/2, 5/2, neighbor counts below and above 32
(both per-point kernel widths), early points with fewer than m neighbors. At a
size the dense oracle cannot reach (n = 20,000, k = 300) the gradient is
checked against central differences of the GPU's own FP64 VIF NLL, and two
calls agree bit for bit.
"""
import numpy as np
import pytest

import synth
from oracle import gradient as GR
from oracle import neighbors as NB
from tests.gpu_util import dev, lib, log, problem_on_device, torch_cuda

pytestmark = pytest.mark.gpu

CASES = {
    "gneiting_m6_k12": dict(seed=61, n_sites=40, n_times=5, k=12, m=6, kind=1),
    "gm_nu05_m8_k15": dict(seed=62, n_sites=40, n_times=5, k=15, m=8, kind=2, nu=0.5),
    "gm_nu15_m10_k20": dict(seed=63, n_sites=45, n_times=5, k=20, m=10, kind=2, nu=1.5),
    "gm_nu25_m5_k10": dict(seed=64, n_sites=40, n_times=4, k=10, m=5, kind=2, nu=2.5),
    "aniso_m12_k25": dict(seed=65, n_sites=40, n_times=6, k=25, m=12, kind=3),
    "gneiting_m40_k30": dict(seed=66, n_sites=50, n_times=5, k=30, m=40, kind=1),
}


def _problem(spec):
    spec = dict(spec)
    nu = spec.pop("nu", None)
    d = synth.config_small(**spec)
    if nu is not None:
        d["kern"] = dict(d["kern"], nu=nu)
    return d


@pytest.mark.parametrize("name", list(CASES))
def test_vif_gradient_matches_oracle(name):
    torch = torch_cuda()
    vif = lib()
    d = _problem(CASES[name])
    kern = d["kern"]
    X = (d["sx"], d["sy"], d["t"])
    Z = (d["zx"], d["zy"], d["zt"])
    nb = NB.brute_force(kern, *X, d["m"])
    nll_o, g_o = GR.vif_grad(kern, X, d["y"], nb, Z)
    Xd, yd, Zd = problem_on_device(d)
    nll, g = vif.vif_nll_grad_vif(*Xd, yd, kern, d["m"], dev(nb, torch.int32), Zd)
    scale = np.abs(g_o).max()
    err = np.abs(g - g_o).max() / scale
    log(f"[grad vif] {name} n={d['n']} m={d['m']} k={d['k']}: nll {nll:.12g} oracle {nll_o:.12g}; "
        f"max grad err / max|g| {err:.3e}")
    assert abs(nll - nll_o) <= 1e-10 * abs(nll_o)
    assert err <= 1e-8, (g, g_o)
    # the NLL is vif_nll's in FP64
    assert abs(nll - vif.vif_nll(*Xd, yd, kern, d["m"], dev(nb, torch.int32), ind=Zd, prec="fp64")) \
        <= 1e-12 * abs(nll)


def test_vif_gradient_at_scale_against_finite_differences():
    torch = torch_cuda()
    vif = lib()
    # k = 300 (kpad 320): the GEMMs span several 128-wide tiles, so the skipped
    # triangular blocks of L_k^-1 and of Gamma'U are exercised
    d = synth.config_small(seed=67, n_times=10, k=300, m=20, kind=1, n_stations=2200)
    kern = d["kern"]
    Xd, yd, Zd = problem_on_device(d)
    nb = vif.vif_neighbors(*Xd, kern, d["m"])
    nll, g = vif.vif_nll_grad_vif(*Xd, yd, kern, d["m"], nb, Zd)
    nll2, g2 = vif.vif_nll_grad_vif(*Xd, yd, kern, d["m"], nb, Zd)
    # Gamma's rows are summed in slot order (no floating-point atomics): repeats agree
    assert nll2 == nll and np.array_equal(g2, g)
    names = GR.PARAMS[kern["kind"]]
    fd = []
    for name in names:
        h = 1e-5 * max(abs(kern[name]), 1e-3)
        kp, km = dict(kern), dict(kern)
        kp[name] += h
        km[name] -= h
        fp = vif.vif_nll(*Xd, yd, kp, d["m"], nb, ind=Zd, prec="fp64")
        fm = vif.vif_nll(*Xd, yd, km, d["m"], nb, ind=Zd, prec="fp64")
        fd.append((fp - fm) / (2 * h))
    fd = np.array(fd)
    err = np.abs(g - fd).max() / np.abs(fd).max()
    log(f"[grad vif] n={d['n']} k={d['k']} m={d['m']}: max |g - fd| / max|fd| {err:.3e}")
    assert err <= 1e-5, (g, fd)
