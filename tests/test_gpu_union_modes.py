"""VIF NLL with hand-built neighbor rows that drive the per-point kernel's union of a
group's conditioning rows to its extremes, against the FP64 oracle.

The NLL is defined for any valid conditioning sets (earlier points, Sec. "Vecchia
approximation"); the rows here are not the correlation-based ones, so that:

* "shared": every point conditions on the same first m points, and a group's union
  is those m rows plus its own points (about m + 8 rows: the widest staged chunks);
* "recent": m distinct random points among the 4m preceding ones (unions of about a
  hundred rows);
* "random": m distinct random earlier points anywhere (unions near the 8 (m + 1)
  maximum: the largest staging buffer);
* "random_wide": the same over more than 16384 points, so that a group's rows span
  an index range too wide for the union's bitmap (the sorting path).

Bars as in test_gpu_parity: FP64 within 1e-8 relative, FP32 and the split-BF16 modes
within 1e-5 relative.
"""
import functools

import numpy as np
import pytest

import synth
from oracle import likelihood as LK
from tests.gpu_util import dev, lib, log, problem_on_device, rel, torch_cuda

pytestmark = pytest.mark.gpu

NLL_TOL = {"fp64": 1e-8, "fp32": 1e-5, "bf16x3": 1e-5, "bf16x6": 1e-5}


def _rows(n, m, mode, seed):
    rng = np.random.default_rng(seed)
    nbr = np.full((n, m), -1, dtype=np.int32)
    for i in range(1, n):
        c = min(i, m)
        if mode == "shared":
            nbr[i, :c] = np.arange(c)
        elif mode == "recent":
            lo = max(0, i - 4 * m)
            nbr[i, :c] = rng.choice(np.arange(lo, i), size=c, replace=False)
        else:
            nbr[i, :c] = rng.choice(i, size=c, replace=False)
    return nbr


@functools.lru_cache(maxsize=None)
def _case(mode):
    """The problem, its neighbor rows and the oracle's result (shared by the precisions)."""
    if mode == "random_wide":
        d = synth.config_small(seed=8, n_times=40, k=30, m=30, kind=1, n_stations=480)
        assert d["n"] > 16384
    else:
        d = synth.config_small(seed=7, n_times=6, k=100, m=30, kind=1, n_stations=300)
    nb = _rows(d["n"], d["m"], "random" if mode == "random_wide" else mode, seed=11)
    o = LK.vif(d["kern"], (d["sx"], d["sy"], d["t"]), d["y"], nb, (d["zx"], d["zy"], d["zt"]))
    return d, nb, o


@pytest.mark.parametrize("mode", ["shared", "recent", "random", "random_wide"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_nll_with_extreme_unions(mode, prec):
    vif = lib()
    torch = torch_cuda()
    d, nb, o = _case(mode)
    Xd, yd, Zd = problem_on_device(d)
    nll = vif.vif_nll(*Xd, yd, d["kern"], d["m"], dev(nb, torch.int32), ind=Zd, prec=prec)
    err = rel(nll, o["nll"])
    log(f"[union] {mode} {prec} n={d['n']} gpu={nll:.12g} oracle={o['nll']:.12g} rel={err:.3e}")
    assert err <= NLL_TOL[prec]


@functools.lru_cache(maxsize=None)
def _case_m(m, mode):
    d = synth.config_small(seed=9, n_times=6, k=60, m=m, kind=1, n_stations=200)
    nb = _rows(d["n"], d["m"], mode, seed=13)
    o = LK.vif(d["kern"], (d["sx"], d["sy"], d["t"]), d["y"], nb, (d["zx"], d["zy"], d["zt"]))
    return d, nb, o


@pytest.mark.parametrize("m", [16, 31])
@pytest.mark.parametrize("mode", ["shared", "random"])
@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_nll_at_the_row_bounds(m, mode, prec):
    """m = 16 and m = 31: the smallest and largest neighbor counts of the 32-row blocks."""
    vif = lib()
    torch = torch_cuda()
    d, nb, o = _case_m(m, mode)
    Xd, yd, Zd = problem_on_device(d)
    nll = vif.vif_nll(*Xd, yd, d["kern"], d["m"], dev(nb, torch.int32), ind=Zd, prec=prec)
    err = rel(nll, o["nll"])
    log(f"[union] m={m} {mode} {prec} n={d['n']} gpu={nll:.12g} oracle={o['nll']:.12g} rel={err:.3e}")
    assert err <= NLL_TOL[prec]


@functools.lru_cache(maxsize=None)
def _case_small_k(mode):
    d = synth.config_small(seed=10, n_times=5, k=20, m=30, kind=1, n_stations=200)
    nb = _rows(d["n"], d["m"], mode, seed=17)
    o = LK.vif(d["kern"], (d["sx"], d["sy"], d["t"]), d["y"], nb, (d["zx"], d["zy"], d["zt"]))
    return d, nb, o


@pytest.mark.parametrize("mode", ["shared", "random"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_nll_with_one_chunk_rows(mode, prec):
    """k = 20: rows of U padded to 64 columns, a single staged chunk (or two) per pass."""
    vif = lib()
    torch = torch_cuda()
    d, nb, o = _case_small_k(mode)
    Xd, yd, Zd = problem_on_device(d)
    nll = vif.vif_nll(*Xd, yd, d["kern"], d["m"], dev(nb, torch.int32), ind=Zd, prec=prec)
    err = rel(nll, o["nll"])
    log(f"[union] k=20 {mode} {prec} n={d['n']} gpu={nll:.12g} oracle={o['nll']:.12g} rel={err:.3e}")
    assert err <= NLL_TOL[prec]
