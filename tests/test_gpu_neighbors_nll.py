"""The combined neighbor search + NLL entry point (vif_neighbors_nll): the search
runs on a library stream beside the low-rank stages, and its neighbor lists and
NLL must be bit-identical to vif_neighbors followed by vif_nll, which are
checked against the oracle elsewhere; the FP64 NLL is also checked against the
oracle here. Errors found on either stream are reported, and the next call works.
"""
import numpy as np
import pytest

import synth
from oracle import likelihood as LK
from oracle import neighbors as NB
from tests.gpu_util import dev, lib, log, problem_on_device, rel, torch_cuda

pytestmark = pytest.mark.gpu

CASES = {
    "gneit_k40_m12": dict(seed=61, n_sites=150, n_times=6, k=40, m=12, kind=1),
    "stations_k60_m30": dict(seed=62, n_times=5, k=60, m=30, kind=1, n_stations=250),
    "aniso_k70_m20": dict(seed=63, n_sites=100, n_times=7, k=70, m=20, kind=3),
    "gneitmatern_k0_m10": dict(seed=64, n_sites=130, n_times=5, k=0, m=10, kind=2),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_combined_equals_separate_calls(name, prec):
    torch = torch_cuda()
    vif = lib()
    d = synth.config_small(**CASES[name])
    Xd, yd, Zd = problem_on_device(d)
    m = d["m"]
    nll, nb = vif.vif_neighbors_nll(*Xd, yd, d["kern"], m, ind=Zd, prec=prec)
    want_nb = vif.vif_neighbors(*Xd, d["kern"], m)
    want = vif.vif_nll(*Xd, yd, d["kern"], m, want_nb, ind=Zd, prec=prec)
    log(f"[combined] {name} {prec}: nll {nll:.12g}")
    assert torch.equal(nb, want_nb)
    assert nll == want
    nll2, nb2 = vif.vif_neighbors_nll(*Xd, yd, d["kern"], m, nbr=nb, ind=Zd, prec=prec)
    assert nll2 == nll and torch.equal(nb2, want_nb)
    if prec == "fp64":
        X = (d["sx"], d["sy"], d["t"])
        nbr = NB.brute_force(d["kern"], *X, m)
        assert np.array_equal(nb.cpu().numpy(), nbr)
        if d["k"]:
            o = LK.vif(d["kern"], X, d["y"], nbr, (d["zx"], d["zy"], d["zt"]))
        else:
            o = LK.vecchia(d["kern"], X, d["y"], nbr)
        assert rel(nll, o["nll"]) <= 1e-10


def test_m_zero_is_the_plain_nll():
    torch = torch_cuda()
    vif = lib()
    d = synth.config_small(seed=65, n_sites=60, n_times=4, k=20, m=5, kind=1)
    Xd, yd, Zd = problem_on_device(d)
    nll, nb = vif.vif_neighbors_nll(*Xd, yd, d["kern"], 0, ind=Zd, prec="fp64")
    assert nb.shape == (d["n"], 0)
    assert nll == vif.vif_nll(*Xd, yd, d["kern"], 0, None, ind=Zd, prec="fp64")


def test_errors_on_either_stream_then_recovery():
    torch = torch_cuda()
    vif = lib()
    d = synth.config_small(seed=66, n_sites=40, n_times=3, k=6, m=4, kind=1)
    Xd, yd, Zd = problem_on_device(d)
    # times out of order: refused by the search before anything is launched
    t = d["t"].copy()
    t[7] += 0.5
    assert t[8] < t[7]
    with pytest.raises(vif.VifError) as e:
        vif.vif_neighbors_nll(Xd[0], Xd[1], dev(t, torch.float64), yd, d["kern"], d["m"], ind=Zd)
    assert e.value.status == 1 and "nondecreasing" in e.value.message
    # Sigma_k not positive definite: found on the NLL stream while the search runs
    zx, zy, zt = d["zx"].copy(), d["zy"].copy(), d["zt"].copy()
    zx[1], zy[1], zt[1] = zx[0], zy[0], zt[0]
    Z = (dev(zx, torch.float64), dev(zy, torch.float64), dev(zt, torch.float64))
    with pytest.raises(vif.VifError) as e:
        vif.vif_neighbors_nll(*Xd, yd, d["kern"], d["m"], ind=Z)
    assert e.value.status == 2 and "Sigma_k" in e.value.message
    nll, nb = vif.vif_neighbors_nll(*Xd, yd, d["kern"], d["m"], ind=Zd, prec="fp64")
    assert nll == vif.vif_nll(*Xd, yd, d["kern"], d["m"], vif.vif_neighbors(*Xd, d["kern"], d["m"]),
                              ind=Zd, prec="fp64")


def test_on_a_side_torch_stream():
    """Caller's stream other than the default one (the library's streams fork from
    and join it; on the null stream the NLL's work runs on a library stream):
    results unchanged."""
    torch = torch_cuda()
    vif = lib()
    d = synth.config_small(**CASES["gneit_k40_m12"])
    Xd, yd, Zd = problem_on_device(d)
    want, want_nb = vif.vif_neighbors_nll(*Xd, yd, d["kern"], d["m"], ind=Zd, prec="bf16x3")
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        got, nb = vif.vif_neighbors_nll(*Xd, yd, d["kern"], d["m"], ind=Zd, prec="bf16x3", stream=st)
    torch.cuda.synchronize()
    assert got == want and torch.equal(nb, want_nb)
