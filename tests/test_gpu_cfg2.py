"""The simulation-scale VIF workload (5000 sites uniform on [0,1]^2 x 20 days,
n = 100,000, m = 30, k = 500 kMeans++ inducing points, Gneiting kernel) against
the FP64 oracle, at full size.

Expected values come from tests/golden/oracle_cfg2.json, written by
tests/golden/make_goldens.py from oracle.neighbors.lag_pruned and
oracle.likelihood.vif alone (FP64, every point). Checked here:
  * every neighbor row bit for bit (SHA-256 of the whole int32 array and of
    each 65,536-row block), and 20,000 sampled rows plus rows 0..m directly
    against the oracle;
  * the FP64 NLL within 1e-8 relative and its four terms;
  * FP64 B and D on 2,000 sampled points within 1e-9 relative + 1e-12 absolute
    (the oracle's per-point VIF factor on those points);
  * FP32 and both split-BF16 NLL within 1e-5 of the oracle. For every
    reduced precision the errors max|dD|/D and max|dB| on the sampled points
    and the relative error of each term (log det M among them) are reported.
This run reaches what the small cases do not: several 4096-row chunks of the
split-BF16 Gram of W, the 1024-row FP32 flushes, and a kpad = 512 Cholesky of M.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import synth
from oracle import likelihood as LK
from oracle import neighbors as NB
from tests.gpu_util import lib, log, problem_on_device, rel, torch_cuda

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_cfg2.json")
NLL_TOL = {"fp64": 1e-8, "fp32": 1e-5, "bf16x6": 1e-5, "bf16x3": 1e-5}


@pytest.fixture(scope="module")
def work():
    torch = torch_cuda()
    vif = lib()
    with open(GOLDEN) as f:
        gold = json.load(f)
    d = synth.config_cfg2()
    assert d["n"] == gold["n"] and d["k"] == gold["k"] and d["m"] == gold["m"]
    log(f"[cfg2] generated {d['name']}")
    Xd, yd, Zd = problem_on_device(d)
    nbr = vif.vif_neighbors(*Xd, d["kern"], d["m"])
    torch.cuda.synchronize()
    rng = np.random.default_rng(21)
    rows = np.sort(np.concatenate([np.arange(0, 40), rng.choice(np.arange(40, d["n"]), 1960, replace=False)]))
    return {"d": d, "gold": gold, "X": Xd, "y": yd, "Z": Zd, "nbr": nbr, "rows": rows, "cache": {}}


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def test_neighbors_every_row(work):
    d, gold = work["d"], work["gold"]
    got = work["nbr"].cpu().numpy()
    br = gold["nbr_block_rows"]
    bad = [b for b, h in enumerate(gold["nbr_block_sha256"]) if _sha(got[b * br:(b + 1) * br]) != h]
    if bad:
        # name the first differing rows of the first differing block
        b = bad[0]
        rows = np.arange(b * br, min((b + 1) * br, d["n"]))[:2000]
        want = NB.lag_pruned(d["kern"], d["sx"], d["sy"], d["t"], d["m"], rows=rows)
        diff = rows[np.nonzero((got[rows] != want).any(1))[0]]
        pytest.fail(f"blocks {bad} differ; first differing rows {diff[:5]}")
    assert _sha(got) == gold["nbr_sha256"]
    log(f"[cfg2] all {d['n']} neighbor rows equal the oracle's (hash)")


def test_neighbors_sampled_rows_direct(work):
    d = work["d"]
    rng = np.random.default_rng(22)
    rows = np.unique(np.concatenate([np.arange(d["m"] + 1), rng.choice(d["n"], 20000, replace=False)]))
    want = NB.lag_pruned(d["kern"], d["sx"], d["sy"], d["t"], d["m"], rows=rows)
    got = work["nbr"].cpu().numpy()[rows]
    bad = np.nonzero((got != want).any(1))[0]
    log(f"[cfg2] neighbors: {rows.shape[0]} rows against the oracle, {bad.size} differ")
    assert bad.size == 0


def _oracle_points(work):
    if "pts" not in work["cache"]:
        d, rows = work["d"], work["rows"]
        X = (d["sx"], d["sy"], d["t"])
        Z = (d["zx"], d["zy"], d["zt"])
        nbr = work["nbr"].cpu().numpy()
        Lk = LK.low_rank_factor(d["kern"], Z)
        work["cache"]["pts"] = LK.vif_points(d["kern"], X, d["y"], nbr, Z, Lk, rows, want_w=False)
    return work["cache"]["pts"]


def test_fp64_factor_sampled_points(work):
    vif = lib()
    d, rows = work["d"], work["rows"]
    B, D = vif.vif_factor(*work["X"], d["kern"], d["m"], work["nbr"], ind=work["Z"], prec="fp64")
    o = _oracle_points(work)
    Dg, Bg = D.cpu().numpy()[rows], B.cpu().numpy()[rows]
    eD = np.max(np.abs(Dg - o["D"]) / o["D"])
    eB = np.max(np.abs(Bg + o["A"]))
    log(f"[cfg2] fp64 factor at {rows.shape[0]} points: max rel err D {eD:.3e}, max abs err B {eB:.3e}")
    np.testing.assert_allclose(Dg, o["D"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Bg, -o["A"], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "bf16x3"])
def test_nll_against_oracle(work, prec):
    vif = lib()
    d, gold = work["d"], work["gold"]
    nll, terms = vif.vif_nll_terms(*work["X"], work["y"], d["kern"], d["m"], work["nbr"],
                                   ind=work["Z"], prec=prec)
    err = rel(nll, gold["nll"])
    names = ("sum_logD", "zz", "logdetM", "quadM")
    terr = {k: rel(v, gold[k]) for k, v in zip(names, terms)}
    msg = f"[cfg2] nll {prec} = {nll:.12g} vs oracle {gold['nll']:.12g}: rel {err:.3e}; " + \
          ", ".join(f"{k} rel {v:.2e}" for k, v in terr.items())
    if prec != "fp64":
        B, D = vif.vif_factor(*work["X"], d["kern"], d["m"], work["nbr"], ind=work["Z"], prec=prec)
        o = _oracle_points(work)
        rows = work["rows"]
        eD = np.max(np.abs(D.cpu().numpy()[rows] - o["D"]) / o["D"])
        eB = np.max(np.abs(B.cpu().numpy()[rows] + o["A"]))
        msg += f"; sampled max|dD|/D {eD:.2e}, max|dB| {eB:.2e}"
    log(msg)
    assert err <= NLL_TOL[prec]
    if prec == "fp64":
        for k, v in terr.items():
            assert v <= 1e-8, (k, v)
