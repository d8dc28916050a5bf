"""vif_neighbors_noalloc (workspace in the library's static device scratch)
against vif_neighbors (caller-owned workspace), through the C ABI.

Two calls in a row on one GPU, the second with a smaller input, so that the
second call runs on what the first left in the shared scratch: both must give
the same rows as vif_neighbors, bit for bit (integer output).
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import lib, log, problem_on_device, torch_cuda

pytestmark = pytest.mark.gpu


def _pair(d):
    torch = torch_cuda()
    vif = lib()
    X, _, _ = problem_on_device(d)
    want = vif.vif_neighbors(*X, d["kern"], d["m"])
    got = torch.full((d["n"], d["m"]), -7, dtype=torch.int32, device="cuda")
    vif.vif_neighbors_noalloc(*X, d["kern"], d["m"], got)
    torch.cuda.synchronize()
    return want.cpu().numpy(), got.cpu().numpy()


def test_noalloc_matches_workspace_call_twice():
    big = synth.config_small(seed=11, n_times=12, k=0, m=30, kind=1, n_stations=2000)
    small = synth.config_small(seed=12, n_sites=150, n_times=6, k=0, m=12, kind=3)
    assert small["n"] < big["n"]
    for name, d in (("big", big), ("small", small)):
        log(f"[noalloc] {name} n={d['n']} m={d['m']} kind={d['kern']['kind']}")
        want, got = _pair(d)
        bad = np.nonzero((got != want).any(1))[0]
        assert bad.size == 0, f"{name}: {bad.size} rows differ, first {bad[:5]}"


def test_noalloc_rejects_too_large_n():
    vif = lib()
    torch = torch_cuda()
    d = synth.config_small(seed=13, n_sites=40, n_times=3, k=0, m=5, kind=1)
    X, _, _ = problem_on_device(d)
    import ctypes
    import paper_2602_03609_amd._lib as L
    p = L.make_points(*X)
    p.n = 50_000_000  # beyond the static scratch; rejected before any launch
    K = L.make_kernel(d["kern"])
    nbr = torch.empty((d["n"], 5), dtype=torch.int32, device="cuda")
    st = L.load().vif_neighbors_noalloc(ctypes.byref(p), ctypes.byref(K), 5, nbr.data_ptr(), None)
    assert st == L.VIF_E_WORKSPACE
    assert b"static scratch" in L.load().vif_last_error()
