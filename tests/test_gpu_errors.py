"""Failure handling through the C ABI on the GPU: conditions are forced from the
host side (inputs), and every kernel still exits normally."""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, lib, problem_on_device, torch_cuda

pytestmark = pytest.mark.gpu


def test_duplicate_points_without_nugget_is_not_pd():
    vif = lib()
    torch = torch_cuda()
    # With one neighbor the conditioning block of point 5 is [[1, 1], [1, 1]]
    # exactly (sigma2 = 1, a duplicate of point 3 at the same time), so its
    # last pivot is exactly zero.
    d = synth.config_small(seed=6, n_sites=40, n_times=3, k=0, m=1, kind=1)
    d["sx"][5] = d["sx"][3]
    d["sy"][5] = d["sy"][3]
    d["t"][5] = d["t"][3]
    kern = dict(d["kern"], nugget=0.0, sigma2=1.0)
    Xd, yd, _ = problem_on_device(d)
    nbr = vif.vif_neighbors(*Xd, kern, d["m"])
    with pytest.raises(vif.VifError) as e:
        vif.vif_nll(*Xd, yd, kern, d["m"], nbr)
    assert e.value.status == 2 and "point 5" in e.value.message


def test_bad_neighbor_rows_are_rejected():
    vif = lib()
    torch = torch_cuda()
    d = synth.config_small(seed=6, n_sites=40, n_times=3, k=0, m=4, kind=1)
    Xd, yd, _ = problem_on_device(d)
    nbr = vif.vif_neighbors(*Xd, d["kern"], d["m"]).cpu().numpy()
    bad = nbr.copy()
    bad[10, 1] = 11            # not an earlier point
    with pytest.raises(vif.VifError) as e:
        vif.vif_nll(*Xd, yd, d["kern"], d["m"], dev(bad, torch.int32))
    assert e.value.status == 1 and "10" in e.value.message
    bad = nbr.copy()
    bad[12, 0] = -1            # padding before a valid entry
    with pytest.raises(vif.VifError):
        vif.vif_factor(*Xd, d["kern"], d["m"], dev(bad, torch.int32))
    bad = nbr.copy()
    bad[15, 2] = 10 ** 6       # out of range
    with pytest.raises(vif.VifError):
        vif.vif_nll(*Xd, yd, d["kern"], d["m"], dev(bad, torch.int32))


def test_unsorted_times_are_rejected_and_fractional_times_searched():
    vif = lib()
    torch = torch_cuda()
    from oracle import neighbors as NB
    d = synth.config_small(seed=6, n_sites=40, n_times=3, k=0, m=4, kind=1)
    Xd, yd, _ = problem_on_device(d)
    t = d["t"].copy()
    t[[0, -1]] = t[[-1, 0]]
    with pytest.raises(vif.VifError) as e:
        vif.vif_neighbors(Xd[0], Xd[1], dev(t, torch.float64), d["kern"], d["m"])
    assert e.value.status == 1
    # one fractional time: the search takes real times (per-pair lag factors)
    t = d["t"] + 0.5 * (np.arange(d["n"]) == 7)
    t = np.maximum.accumulate(t)
    got = vif.vif_neighbors(Xd[0], Xd[1], dev(t, torch.float64), d["kern"], d["m"]).cpu().numpy()
    want = NB.brute_force(d["kern"], d["sx"], d["sy"], t, d["m"])
    assert np.array_equal(got, want)
    # the proposal search keeps to integer times
    E = torch.zeros((d["n"], 16), dtype=torch.float32, device="cuda")
    with pytest.raises(vif.VifError) as e:
        vif.vif_propose_neighbors(Xd[0], Xd[1], dev(t, torch.float64), d["kern"], d["m"], E, 8, 0.2, 1,
                                  64, wmin=10, rmax=3)
    assert e.value.status == 5


def test_sigma_k_not_pd_is_reported():
    vif = lib()
    torch = torch_cuda()
    d = synth.config_small(seed=6, n_sites=40, n_times=3, k=6, m=4, kind=1)
    zx, zy, zt = d["zx"].copy(), d["zy"].copy(), d["zt"].copy()
    zx[1], zy[1], zt[1] = zx[0], zy[0], zt[0]   # duplicate: second pivot exactly 0
    Xd, yd, _ = problem_on_device(d)
    Z = (dev(zx, torch.float64), dev(zy, torch.float64), dev(zt, torch.float64))
    nbr = vif.vif_neighbors(*Xd, d["kern"], d["m"])
    with pytest.raises(vif.VifError) as e:
        vif.vif_nll(*Xd, yd, d["kern"], d["m"], nbr, ind=Z)
    assert e.value.status == 2 and "Sigma_k" in e.value.message
    # a small jitter repairs it when the caller asks for one
    kern = dict(d["kern"], jitter=1e-6)
    vif.vif_nll(*Xd, yd, kern, d["m"], nbr, ind=Z)
