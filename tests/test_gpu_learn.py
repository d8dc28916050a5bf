"""GPU kernels of the learned neighbor proposal (through the C ABI) against the
FP64 oracle: features, network forward and backward, contrastive loss, Adam,
batch assembly, and the proposal search (bit-exact, both candidate modes).

Bars: features within 1e-7 relative (FP32 rounding of FP64 values); forward
within 2e-5 of the largest embedding entry (FP32 sums of 64 terms); gradients
within 1e-4 of the largest gradient entry (FP32 sums over rows); loss within
1e-5 relative; Adam within 1e-6; proposal rows bit-exact (the FP32 embedding
distance is taken in the same order and precision on both sides).
"""
import numpy as np
import pytest

import synth
from oracle import learn as LR
from oracle import neighbors as NB
from tests.gpu_util import dev, lib, log, problem_on_device, torch_cuda

pytestmark = pytest.mark.gpu

CENTRE = [0.5, 0.5, 3.0, 0.3, 2.0, 0.0, 3.0, -0.3, -0.7, -0.7]


def _params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(scale=scale, size=LR.N_PARAMS)


def test_features_match_oracle():
    torch = torch_cuda()
    vif = lib()
    d = synth.config_small(seed=11, n_sites=80, n_times=5, k=0, m=8)
    kern = synth.perturb_hyper(d["kern"], np.random.default_rng(11))
    X, _, _ = problem_on_device(d)
    got = vif.vif_mlp_features(*X, kern, CENTRE).cpu().numpy()
    want = LR.features(d["sx"], d["sy"], d["t"], kern, CENTRE)
    assert np.allclose(got, want.astype(np.float32), rtol=1e-7, atol=1e-7)


@pytest.mark.parametrize("rows", [1, 63, 64, 200, 1000])
def test_forward_backward_match_oracle(rows):
    torch = torch_cuda()
    vif = lib()
    rng = np.random.default_rng(rows)
    p = _params(rows)
    Xn = rng.normal(size=(rows, 8))
    dEn = rng.normal(size=(rows, 16))
    P = dev(p, torch.float32)
    Xd = dev(Xn, torch.float32)
    E, H = vif.vif_mlp_forward(P, Xd, want_hidden=True)
    p32 = p.astype(np.float32).astype(np.float64)
    X32 = Xn.astype(np.float32).astype(np.float64)
    Ew, cache = LR.forward(p32, X32)
    err = np.abs(E.cpu().numpy() - Ew).max() / np.abs(Ew).max()
    log(f"forward rows={rows}: max err {err:.2e}")
    assert err < 2e-5
    assert np.allclose(H.cpu().numpy()[:, 0, :], cache[1], atol=1e-4 * np.abs(cache[1]).max())
    g = vif.vif_mlp_backward(P, Xd, H, dev(dEn, torch.float32)).cpu().numpy()
    gw = LR.backward(p32, cache, dEn.astype(np.float32).astype(np.float64))
    gerr = np.abs(g - gw).max() / np.abs(gw).max()
    log(f"backward rows={rows}: max err {gerr:.2e}")
    assert gerr < 1e-4


def test_backward_is_deterministic():
    torch = torch_cuda()
    vif = lib()
    rng = np.random.default_rng(5)
    P = dev(_params(5), torch.float32)
    Xd = dev(rng.normal(size=(3000, 8)), torch.float32)
    E, H = vif.vif_mlp_forward(P, Xd, want_hidden=True)
    dE = dev(rng.normal(size=(3000, 16)), torch.float32)
    g1 = vif.vif_mlp_backward(P, Xd, H, dE)
    g2 = vif.vif_mlp_backward(P, Xd, H, dE)
    assert torch.equal(g1, g2)


@pytest.mark.parametrize("npos,nneg", [(1, 1), (30, 30), (30, 46), (5, 3)])
def test_pair_loss_matches_oracle(npos, nneg):
    torch = torch_cuda()
    vif = lib()
    rng = np.random.default_rng(npos * 100 + nneg)
    G = 1 + npos + nneg
    En = rng.normal(size=(17 * G, 16)).astype(np.float32)
    loss, dE = vif.vif_mlp_pair_loss(dev(En), npos, nneg, 0.8)
    lw, dw = LR.pair_loss(En.astype(np.float64), npos, nneg, 0.8)
    assert np.allclose(loss.cpu().numpy(), lw, rtol=1e-5, atol=1e-6)
    assert np.abs(dE.cpu().numpy() - dw).max() <= 1e-5 * np.abs(dw).max()


def test_adam_matches_oracle():
    torch = torch_cuda()
    vif = lib()
    rng = np.random.default_rng(9)
    p = rng.normal(size=1000)
    m = rng.normal(size=1000) * 0.1
    v = np.abs(rng.normal(size=1000)) * 0.01
    g = rng.normal(size=1000)
    P, M, V = (dev(a, torch.float32) for a in (p, m, v))
    vif.vif_mlp_adam(P, dev(g, torch.float32), M, V, 7, 1e-3)
    pw, mw, vw = LR.adam(p, g, m, v, 7, 1e-3)
    assert np.allclose(P.cpu().numpy(), pw, atol=1e-6)
    assert np.allclose(M.cpu().numpy(), mw, atol=1e-6) and np.allclose(V.cpu().numpy(), vw, atol=1e-6)


def test_batch_rows():
    torch = torch_cuda()
    vif = lib()
    rng = np.random.default_rng(3)
    n, m_ext = 500, 12
    Xn = rng.normal(size=(n, 8)).astype(np.float32)
    nbr = np.stack([rng.choice(i, m_ext, replace=False) if i >= m_ext else np.zeros(m_ext, int)
                    for i in range(n)]).astype(np.int32)
    q = np.array([100, 250, 499], dtype=np.int32)
    rnd = rng.integers(0, 2**31 - 1, size=(3, 4)).astype(np.int32)
    Xb = vif.vif_mlp_batch(dev(Xn), dev(q), dev(nbr), 5, 3, 4, dev(rnd), 50).cpu().numpy()
    G = 1 + 5 + 3 + 4
    for b, qq in enumerate(q):
        rows = [qq] + list(nbr[qq, :8])
        for r in range(4):
            j = qq - 1 - (int(np.uint32(rnd[b, r])) % min(int(qq), 50))
            if j in nbr[qq, :8]:
                j = nbr[qq, 7]
            rows.append(j)
        assert np.array_equal(Xb[b * G:(b + 1) * G], Xn[rows])


CASES = {
    "grid_m8": lambda: synth.config_small(seed=21, n_sites=150, n_times=6, k=0, m=8),
    "stations_m30": lambda: synth.config_small(seed=22, n_times=6, k=0, m=30, n_stations=400),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("use_e", [False, True])
@pytest.mark.parametrize("adaptive", [False, True])
def test_propose_matches_oracle(name, use_e, adaptive):
    torch = torch_cuda()
    vif = lib()
    d = CASES[name]()
    X, _, _ = problem_on_device(d)
    n, m, kern = d["n"], d["m"], d["kern"]
    span_x = d["sx"].max() - d["sx"].min()
    cell = span_x / (20.0 if adaptive else 7.0)
    wmin, rmax = (4 * m, 9) if adaptive else (0, 1)
    E = np.random.default_rng(1).normal(size=(n, 16)).astype(np.float32) if use_e else None
    ncand, lags, cmax = min(4 * m, 128), 1, 600
    got, nfb = vif.vif_propose_neighbors(*X, kern, m, dev(E) if use_e else None, ncand, cell,
                                         lags, cmax, wmin=wmin, rmax=rmax)
    want, fb = LR.propose(kern, d["sx"], d["sy"], d["t"], m, E, ncand, cell, lags, cmax,
                          wmin=wmin, rmax=rmax)
    log(f"propose {name} E={use_e} adaptive={adaptive}: fallback {nfb} (oracle {int(fb.sum())})")
    assert nfb == int(fb.sum())
    assert np.array_equal(got.cpu().numpy(), want)


def test_propose_full_window_equals_exact_search():
    torch = torch_cuda()
    vif = lib()
    d = synth.config_small(seed=23, n_sites=30, n_times=4, k=0, m=10)
    X, _, _ = problem_on_device(d)
    got, nfb = vif.vif_propose_neighbors(*X, d["kern"], d["m"], None, 128, 1e9,
                                         int(d["t"][-1] - d["t"][0]), 1024)
    exact = vif.vif_neighbors(*X, d["kern"], d["m"])
    assert torch.equal(got, exact)


def test_trained_network_beats_spatial_candidates():
    """What the network gains: trained on the GPU by the library's own kernels, its
    candidates recover more exact neighbors than the same budget drawn from the same
    window by spatial distance (on a held-out problem)."""
    torch = torch_cuda()
    vif = lib()
    from paper_2602_03609_amd import learn as LN
    m = 30
    train = LN.training_problems(8, n_days=8, m=m)
    params, hist = LN.train(train, steps=2500, log_every=500, log=log)
    ev = synth.config_station_days(seed=100, n_days=8, m=m, day0=120)
    X = tuple(dev(ev[k], torch.float64) for k in ("sx", "sy", "t"))
    exact = vif.vif_neighbors(*X, ev["kern"], m)
    E = LN.embed(params, X, ev["kern"])
    args = dict(wmin=480, rmax=30)
    learned, _ = vif.vif_propose_neighbors(*X, ev["kern"], m, E, 120, 50.0, 1, 1024, **args)
    spatial, _ = vif.vif_propose_neighbors(*X, ev["kern"], m, None, 120, 50.0, 1, 1024, **args)
    r_l, r_s = LN.recall(learned, exact), LN.recall(spatial, exact)
    log(f"held-out recall: learned {r_l:.5f}, spatial candidates {r_s:.5f}")
    assert hist[-1][1] < hist[0][1]
    assert r_l > r_s + 0.01
