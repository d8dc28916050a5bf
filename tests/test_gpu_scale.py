"""GPU path at the benchmark's full size (continental network, n ~ 1.1M, m = 30,
k = 1000), in the launch configuration bench.py times, checked on sampled
outputs the oracle computes one by one, on the oracle's whole-problem values
(tests/golden/oracle_cfg3.json, written by tests/golden/make_goldens.py from
oracle/ alone: the SHA-256 of all neighbor rows and the FP64 NLL with its four
terms), and on properties that hold at any size.
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

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_cfg3.json")
NLL_TOL = {"fp64": 1e-8, "fp32": 1e-5, "bf16x6": 1e-5, "bf16x3": 1e-5}


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


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
    np.testing.assert_allclose(Bg, -o["A"], rtol=1e-9, atol=1e-12)


def test_neighbors_every_row_equals_oracle(big):
    d, Xd, yd, Zd, nbr = big
    gold = _golden()
    assert gold["n"] == d["n"] and gold["m"] == d["m"]
    got = nbr.cpu().numpy()
    br = gold["nbr_block_rows"]
    bad = [b for b, h in enumerate(gold["nbr_block_sha256"]) if _sha(got[b * br:(b + 1) * br]) != h]
    log(f"[scale] neighbors: {len(gold['nbr_block_sha256'])} blocks of {br} rows, {len(bad)} differ")
    if bad:
        b = bad[0]
        rows = np.arange(b * br, min((b + 1) * br, d["n"]))[:1000]
        X = (d["sx"], d["sy"], d["t"])
        want = NB.lag_pruned(d["kern"], *X, d["m"], rows=rows)
        diff = rows[np.nonzero((got[rows] != want).any(1))[0]]
        pytest.fail(f"blocks {bad} differ; first differing rows {diff[:5]}")
    assert _sha(got) == gold["nbr_sha256"]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "bf16x3"])
def test_nll_against_oracle_golden(big, prec):
    """Whole-problem NLL against the oracle's FP64 value; for the reduced
    precisions also max|dD|/D and max|dB| on sampled points and the relative
    error of log det M."""
    vif = lib()
    d, Xd, yd, Zd, nbr = big
    gold = _golden()
    nll, terms = vif.vif_nll_terms(*Xd, yd, d["kern"], d["m"], nbr, ind=Zd, prec=prec)
    err = rel(nll, gold["nll"])
    names = ("sum_logD", "zz", "logdetM", "quadM")
    terr = {k: rel(v, gold[k]) for k, v in zip(names, terms)}
    msg = (f"[scale] nll {prec} = {nll:.12g} vs oracle {gold['nll']:.12g}: rel {err:.3e}; "
           + ", ".join(f"{k} rel {v:.2e}" for k, v in terr.items()))
    if prec != "fp64":
        B, D = vif.vif_factor(*Xd, d["kern"], d["m"], nbr, ind=Zd, prec=prec)
        rows, o = _sampled_oracle(d)
        eD = np.max(np.abs(D.cpu().numpy()[rows] - o["D"]) / o["D"])
        eB = np.max(np.abs(B.cpu().numpy()[rows] + o["A"]))
        msg += f"; sampled max|dD|/D {eD:.2e}, max|dB| {eB:.2e}"
        del B, D
    log(msg)
    assert err <= NLL_TOL[prec]
    if prec == "fp64":
        for k, v in terr.items():
            assert v <= 1e-8, (k, v)


_SAMPLED = {}


def _sampled_oracle(d):
    if "o" not in _SAMPLED:
        rng = np.random.default_rng(13)
        rows = np.sort(np.concatenate([np.arange(0, 10), rng.choice(d["n"], 150, replace=False)]))
        X = (d["sx"], d["sy"], d["t"])
        Z = (d["zx"], d["zy"], d["zt"])
        nb_rows = NB.lag_pruned(d["kern"], *X, d["m"], rows=rows)
        nbr_full = np.full((d["n"], d["m"]), -1, dtype=np.int32)
        nbr_full[rows] = nb_rows
        Lk = LK.low_rank_factor(d["kern"], Z)
        _SAMPLED["o"] = (rows, LK.vif_points(d["kern"], X, d["y"], nbr_full, Z, Lk, rows, want_w=False))
    return _SAMPLED["o"]


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
