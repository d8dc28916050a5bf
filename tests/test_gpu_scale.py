"""GPU path at the benchmark's full size (continental network, n ~ 1.1M, m = 30,
k = 1000), in the launch configuration bench.py times, checked on sampled
outputs the oracle computes one by one, and on properties that hold at any size.
"""
import numpy as np
import pytest

import synth
from oracle import likelihood as LK
from oracle import neighbors as NB
from tests.gpu_util import lib, log, problem_on_device, rel, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    torch = torch_cuda()
    vif = lib()
    d = synth.config_cfg3()
    log(f"[scale] generated {d['name']}")
    Xd, yd, Zd = problem_on_device(d)
    nbr = vif.vif_neighbors(*Xd, d["kern"], d["m"])
    torch.cuda.synchronize()
    return d, Xd, yd, Zd, nbr


def test_neighbors_sampled_rows_bit_exact(big):
    d, Xd, yd, Zd, nbr = big
    rng = np.random.default_rng(11)
    rows = np.concatenate([np.arange(0, 40), rng.choice(d["n"], 600, replace=False)])
    X = (d["sx"], d["sy"], d["t"])
    want = NB.lag_pruned(d["kern"], *X, d["m"], rows=rows)
    got = nbr.cpu().numpy()[rows]
    bad = np.nonzero((got != want).any(1))[0]
    log(f"[scale] neighbors: {rows.shape[0]} sampled rows, {bad.size} differ")
    assert bad.size == 0


def test_neighbors_repeatable(big):
    torch = torch_cuda()
    vif = lib()
    d, Xd, yd, Zd, nbr = big
    again = vif.vif_neighbors(*Xd, d["kern"], d["m"])
    assert torch.equal(again, nbr)


def test_vif_factor_sampled_points_fp64(big):
    vif = lib()
    d, Xd, yd, Zd, nbr = big
    B, D = vif.vif_factor(*Xd, d["kern"], d["m"], nbr, ind=Zd, prec="fp64")
    rng = np.random.default_rng(12)
    rows = np.sort(np.concatenate([np.arange(0, 20), rng.choice(d["n"], 300, replace=False)]))
    X = (d["sx"], d["sy"], d["t"])
    Z = (d["zx"], d["zy"], d["zt"])
    nb_rows = NB.lag_pruned(d["kern"], *X, d["m"], rows=rows)
    nbr_full = np.full((d["n"], d["m"]), -1, dtype=np.int32)
    nbr_full[rows] = nb_rows
    Lk = LK.low_rank_factor(d["kern"], Z)
    o = LK.vif_points(d["kern"], X, d["y"], nbr_full, Z, Lk, rows, want_w=False)
    Dg = D.cpu().numpy()[rows]
    Bg = B.cpu().numpy()[rows]
    eD = np.max(np.abs(Dg - o["D"]) / o["D"])
    log(f"[scale] factor fp64 at {rows.shape[0]} sampled points: max rel err D {eD:.3e}")
    np.testing.assert_allclose(Dg, o["D"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Bg, -o["A"], rtol=1e-7, atol=1e-10)


def test_mixed_precision_nll_vs_fp64(big):
    vif = lib()
    d, Xd, yd, Zd, nbr = big
    ref, t64 = vif.vif_nll_terms(*Xd, yd, d["kern"], d["m"], nbr, ind=Zd, prec="fp64")
    errs = {}
    for prec in ("fp32", "bf16x6", "bf16x3"):
        v, tv = vif.vif_nll_terms(*Xd, yd, d["kern"], d["m"], nbr, ind=Zd, prec=prec)
        errs[prec] = rel(v, ref)
        log(f"[scale] nll {prec} = {v:.12g} vs fp64 {ref:.12g}: rel {errs[prec]:.3e}; terms {tv} vs {t64}")
    assert errs["fp32"] <= 1e-5
    assert errs["bf16x6"] <= 1e-5
    assert errs["bf16x3"] <= 1e-4


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
def test_combined_call_matches_separate_calls(big, prec):
    """vif_neighbors_nll, the call bench.py times: neighbor lists and NLL
    bit-identical to the two separate calls at full size."""
    torch = torch_cuda()
    vif = lib()
    d, Xd, yd, Zd, nbr = big
    nll, nb = vif.vif_neighbors_nll(*Xd, yd, d["kern"], d["m"], ind=Zd, prec=prec)
    want = vif.vif_nll(*Xd, yd, d["kern"], d["m"], nbr, ind=Zd, prec=prec)
    log(f"[scale] combined {prec}: nll {nll:.12g} (separate {want:.12g})")
    assert torch.equal(nb, nbr)
    assert nll == want
