"""GPU path (through the C ABI) against the FP64 oracle.

Bars: neighbor sets bit-exact (indices, order, -1 padding); FP64 NLL within
1e-8 relative; FP64 B and D within 1e-9 relative + 1e-12 absolute; FP32 and
both split-BF16 modes (three products, the mixed precision the benchmark
times, and six) NLL within 1e-5 relative.
"""
import numpy as np
import pytest

import synth
from oracle import likelihood as LK
from oracle import neighbors as NB
from tests.gpu_util import dev, lib, log, problem_on_device, rel, torch_cuda

pytestmark = pytest.mark.gpu

NLL_TOL = {"fp64": 1e-8, "fp32": 1e-5, "bf16x6": 1e-5, "bf16x3": 1e-5}


def _cases():
    return {
        "cfg1": lambda: synth.config_cfg1(),
        "gneit_k40_m12": lambda: synth.config_small(seed=1, n_sites=150, n_times=6, k=40, m=12, kind=1),
        "gneitmatern_m5": lambda: synth.config_small(seed=2, n_sites=120, n_times=5, k=30, m=5, kind=2),
        "stations_m30_k100": lambda: synth.config_small(seed=3, n_times=8, k=100, m=30, kind=1,
                                                        n_stations=300),
        "aniso_m40_k70": lambda: synth.config_small(seed=4, n_sites=100, n_times=8, k=70, m=40, kind=3),
    }


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
def test_neighbors_bit_exact(name):
    torch = torch_cuda()
    vif = lib()
    d = CASES[name]()
    log(f"[neighbors] {name} n={d['n']} m={d['m']}")
    X = (d["sx"], d["sy"], d["t"])
    want = NB.brute_force(d["kern"], *X, d["m"])
    Xd, _, _ = problem_on_device(d)
    got = vif.vif_neighbors(*Xd, d["kern"], d["m"]).cpu().numpy()
    torch.cuda.synchronize()
    assert got.shape == want.shape
    bad = np.nonzero((got != want).any(1))[0]
    assert bad.size == 0, f"{bad.size} rows differ, first {bad[:5]}: {got[bad[0]]} vs {want[bad[0]]}"


def test_lowrank_diagonal_matches_oracle():
    """m = 0 with inducing points: D_i = sigma2 + nugget - |U_i|^2 isolates U = C(X,Z) L_k^-T."""
    vif = lib()
    torch = torch_cuda()
    d = synth.config_small(seed=1, n_sites=150, n_times=6, k=40, m=0, kind=1)
    X = (d["sx"], d["sy"], d["t"])
    Xd, _, Zd = problem_on_device(d)
    _, D = vif.vif_factor(*Xd, d["kern"], 0, None, ind=Zd, prec="fp64")
    o = LK.vif(d["kern"], X, d["y"], np.zeros((d["n"], 0), np.int32), (d["zx"], d["zy"], d["zt"]))
    Dg = D.cpu().numpy()
    err = np.max(np.abs(Dg - o["D"]) / np.abs(o["D"]))
    log(f"[lowrank diag] max rel err {err:.3e}; gpu {Dg[:4]} oracle {o['D'][:4]}")
    np.testing.assert_allclose(Dg, o["D"], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("name", list(CASES))
def test_factor_matches_oracle(name):
    vif = lib()
    d = CASES[name]()
    log(f"[factor] {name} n={d['n']} m={d['m']} k={d['k']}")
    X = (d["sx"], d["sy"], d["t"])
    nb = NB.brute_force(d["kern"], *X, d["m"])
    Xd, _, Zd = problem_on_device(d)
    torch = torch_cuda()
    B, D = vif.vif_factor(*Xd, d["kern"], d["m"], dev(nb, torch.int32), ind=Zd, prec="fp64")
    if d["k"]:
        o = LK.vif(d["kern"], X, d["y"], nb, (d["zx"], d["zy"], d["zt"]))
    else:
        o = LK.vecchia(d["kern"], X, d["y"], nb)
    Dg, Bg = D.cpu().numpy(), B.cpu().numpy()
    eD = np.max(np.abs(Dg - o["D"]) / np.abs(o["D"]))
    eB = np.max(np.abs(Bg + o["A"]) / (np.abs(o["A"]) + 1e-3))
    log(f"[factor] {name} max rel err D {eD:.3e}, B {eB:.3e}")
    np.testing.assert_allclose(Dg, o["D"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Bg, -o["A"], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("name", list(CASES))
def test_nll_matches_oracle(name, prec):
    vif = lib()
    torch = torch_cuda()
    d = CASES[name]()
    X = (d["sx"], d["sy"], d["t"])
    nb = NB.brute_force(d["kern"], *X, d["m"])
    Xd, yd, Zd = problem_on_device(d)
    nll, terms = vif.vif_nll_terms(*Xd, yd, d["kern"], d["m"], dev(nb, torch.int32), ind=Zd, prec=prec)
    if d["k"]:
        o = LK.vif(d["kern"], X, d["y"], nb, (d["zx"], d["zy"], d["zt"]))
    else:
        o = LK.vecchia(d["kern"], X, d["y"], nb)
        o["sum_logD"] = float(np.log(o["D"]).sum())
        o["zz"] = float((o["e"] ** 2 / o["D"]).sum())
        o["logdetM"] = o["quadM"] = 0.0
    err = rel(nll, o["nll"])
    log(f"[nll] {name} {prec} gpu={nll:.12g} oracle={o['nll']:.12g} rel={err:.3e} "
        f"terms={terms} oracle_terms={[o['sum_logD'], o['zz'], o['logdetM'], o['quadM']]}")
    assert err <= NLL_TOL[prec]


def test_fitc_and_vecchia_degenerate_cases():
    """m = 0 with inducing points is FITC; k = 0 is plain Vecchia; m = 0, k = 0 is independent."""
    vif = lib()
    torch = torch_cuda()
    d = synth.config_small(seed=5, n_sites=80, n_times=4, k=25, m=0, kind=1)
    X = (d["sx"], d["sy"], d["t"])
    Xd, yd, Zd = problem_on_device(d)
    nb0 = np.zeros((d["n"], 0), dtype=np.int32)
    o = LK.vif(d["kern"], X, d["y"], nb0, (d["zx"], d["zy"], d["zt"]))
    got = vif.vif_nll(*Xd, yd, d["kern"], 0, None, ind=Zd)
    assert rel(got, o["nll"]) <= 1e-8
    o = LK.vecchia(d["kern"], X, d["y"], nb0)
    got = vif.vif_nll(*Xd, yd, d["kern"], 0, None, ind=None)
    assert rel(got, o["nll"]) <= 1e-8


def test_repeatable_bits():
    vif = lib()
    torch = torch_cuda()
    d = CASES["stations_m30_k100"]()
    Xd, yd, Zd = problem_on_device(d)
    nb = vif.vif_neighbors(*Xd, d["kern"], d["m"])
    vals = [vif.vif_nll(*Xd, yd, d["kern"], d["m"], nb, ind=Zd, prec=p) for p in ("fp64",) * 3]
    assert vals[0] == vals[1] == vals[2]
    nb2 = vif.vif_neighbors(*Xd, d["kern"], d["m"])
    assert torch.equal(nb, nb2)
