"""Pins of the learned-proposal oracle (CPU only): the network's gradients
against central finite differences, the loss against closed forms, one Adam
step against its closed form, features by hand, and the proposal search
against the exact search where the window covers every earlier point."""
import math

import numpy as np
import pytest

import synth
from oracle import learn as LR
from oracle import neighbors as NB


def rand_params(rng, scale=0.4):
    return rng.normal(scale=scale, size=LR.N_PARAMS)


def test_parameter_count_and_packing():
    assert LR.N_PARAMS == 9936
    rng = np.random.default_rng(0)
    p = rand_params(rng)
    assert np.array_equal(LR.pack(LR.unpack(p)), p)
    d = LR.unpack(p)
    assert d["W1"].shape == (8, 64) and d["b4"].shape == (16,)
    assert d["W1"][0, 1] == p[1] and d["b1"][0] == p[512]


def test_forward_is_the_layer_composition():
    """A network whose hidden layers are identity maps on the positive orthant
    reduces to an affine map of the input."""
    rng = np.random.default_rng(1)
    d = {k: np.zeros(s) for k, s in LR.SHAPES}
    d["W1"][:, :8] = np.eye(8)
    d["b1"][:8] = 10.0                      # keeps the 8 used units positive
    d["W2"][:8, :8] = np.eye(8)
    d["W3"][:8, :8] = np.eye(8)
    A = rng.normal(size=(8, 16))
    d["W4"][:8, :] = A
    d["b4"][:] = rng.normal(size=16)
    X = rng.uniform(-1, 1, size=(5, 8))
    E, _ = LR.forward(LR.pack(d), X)
    assert np.allclose(E, (X + 10.0) @ A + d["b4"])


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = rand_params(rng)
    X = rng.normal(size=(7, 8))
    dE = rng.normal(size=(7, 16))
    E, cache = LR.forward(p, X)
    g = LR.backward(p, cache, dE)
    f = lambda q: float((LR.forward(q, X)[0] * dE).sum())
    idx = rng.choice(LR.N_PARAMS, 60, replace=False)
    # include biases and every layer
    idx = np.concatenate([idx, [0, 512, 600, 4700, 4900, 9000, 9800, 9935]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        num = (f(p + e) - f(p - e)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num)), (i, num, g[i])


def test_pair_loss_closed_form():
    """One query, one positive, one negative: loss = softplus((d_p - d_n) / tau)."""
    E = np.zeros((3, 16))
    E[1, 0] = 1.0   # d_p = 1
    E[2, 1] = 2.0   # d_n = 4
    for tau in (0.5, 1.0, 3.0):
        loss, dE = LR.pair_loss(E, 1, 1, tau)
        assert math.isclose(loss[0], math.log1p(math.exp(-3.0 / tau)), rel_tol=1e-14)
        s = 1.0 / (1.0 + math.exp(3.0 / tau))          # sigmoid((d_p - d_n)/tau)
        # d_p = |q - e_p|^2: dd_p/de_p = -2 (q - e_p) = (2, 0, ...)
        assert math.isclose(dE[1, 0], s / tau * 2.0, rel_tol=1e-12)
        assert math.isclose(dE[2, 1], -s / tau * 4.0, rel_tol=1e-12)
        assert np.allclose(dE.sum(0), 0.0)             # translation invariance


def test_pair_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    npos, nneg = 3, 4
    E = rng.normal(size=(2 * (1 + npos + nneg), 16))
    loss, dE = LR.pair_loss(E, npos, nneg, 0.7)
    h = 1e-6
    for _ in range(40):
        r, c = rng.integers(E.shape[0]), rng.integers(16)
        Ep, Em = E.copy(), E.copy()
        Ep[r, c] += h
        Em[r, c] -= h
        num = (LR.pair_loss(Ep, npos, nneg, 0.7)[0].sum() - LR.pair_loss(Em, npos, nneg, 0.7)[0].sum()) / (2 * h)
        assert abs(num - dE[r, c]) <= 1e-7 * max(1.0, abs(num))


def test_adam_first_step_is_a_signed_step():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p = np.zeros(4)
    p1, m, v = LR.adam(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-12)
    # bias-corrected m = g and v = g^2, so the step is -lr * g / |g|
    assert np.allclose(p1[:3], -0.01 * np.sign(g[:3]), rtol=1e-9)
    assert p1[3] == 0.0
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_by_hand():
    kern = synth.kern_gneiting(a=2.0, c=0.5, alpha=0.75, beta=0.5, gamma=0.25)
    sx, sy, t = np.array([1.0, 3.0]), np.array([2.0, -2.0]), np.array([0.0, 4.0])
    centre = [1.0, 0.0, 2.0, 2.0, 4.0, 0.0, 0.0, 0.0, 0.0, 0.0]
    X = LR.features(sx, sy, t, kern, centre)
    assert np.allclose(X[0, :3], [0.0, 1.0, -0.5]) and np.allclose(X[1, :3], [1.0, -1.0, 0.5])
    assert np.allclose(X[:, 3:], [math.log(2.0), math.log(0.5), math.log(0.75), math.log(0.5),
                                  math.log(0.25)])


def test_emb_dist32_is_exact_on_small_integers():
    E = np.arange(48, dtype=np.float64).reshape(3, 16) % 7
    d = LR.emb_dist32(E, 0, np.array([1, 2]))
    want = [((E[0] - E[j]) ** 2).sum() for j in (1, 2)]
    assert d.dtype == np.float32 and np.array_equal(d, np.array(want, dtype=np.float32))


def test_window_definition():
    rng = np.random.default_rng(4)
    d = synth.config_small(seed=4, n_sites=60, n_times=5, k=0, m=8)
    sx, sy, t = d["sx"], d["sy"], d["t"]
    cx, cy = LR.grid_cells(sx, sy, 0.2)
    for i in rng.choice(sx.shape[0], 20, replace=False):
        got = LR.window(t, cx, cy, i, 1)
        want = [j for j in range(i) if t[i] - t[j] <= 1 and abs(cx[j] - cx[i]) <= 1
                and abs(cy[j] - cy[i]) <= 1]
        assert list(got) == want


@pytest.mark.parametrize("use_e", [False, True])
def test_full_window_reproduces_the_exact_search(use_e):
    """One grid cell, every lag and ncand >= i: the proposal reranks every earlier
    point with the exact key, which is the brute-force search."""
    d = synth.config_small(seed=5, n_sites=40, n_times=4, k=0, m=6)
    sx, sy, t, m, kern = d["sx"], d["sy"], d["t"], d["m"], d["kern"]
    n = sx.shape[0]
    E = np.random.default_rng(5).normal(size=(n, 16)) if use_e else None
    lags = int(t[-1] - t[0])
    prop, fb = LR.propose(kern, sx, sy, t, m, E, n, 1e9, lags, n)
    assert np.array_equal(prop, NB.brute_force(kern, sx, sy, t, m))
    assert not fb.any()


def test_fallback_rows_take_the_exact_search():
    d = synth.config_small(seed=6, n_sites=50, n_times=4, k=0, m=8)
    sx, sy, t, m, kern = d["sx"], d["sy"], d["t"], d["m"], d["kern"]
    # a tiny cmax sends every row with more than 5 window points to the exact search
    prop, fb = LR.propose(kern, sx, sy, t, m, None, 16, 0.3, 1, 5)
    exact = NB.brute_force(kern, sx, sy, t, m)
    assert fb.any()
    assert np.array_equal(prop[fb], exact[fb])


def test_recall_counts_set_overlap():
    a = np.array([[1, 2, 3, -1], [4, 5, 6, 7]])
    b = np.array([[3, 2, 9, -1], [7, 6, 5, 4]])
    assert LR.recall(a, b) == pytest.approx(6 / 7)
    assert LR.recall(b, b) == 1.0


def test_network_beats_nothing_only_when_trained():
    """Spatial candidates recover most exact neighbors when the window is wide;
    a random embedding does not (the test the trained network has to pass)."""
    d = synth.config_small(seed=7, n_sites=120, n_times=4, k=0, m=8)
    sx, sy, t, m, kern = d["sx"], d["sy"], d["t"], d["m"], d["kern"]
    rows = np.arange(200, sx.shape[0], 7)
    exact = NB.brute_force(kern, sx, sy, t, m, rows=rows)
    sp, _ = LR.propose(kern, sx, sy, t, m, None, 16, 0.25, 1, 4096, rows=rows)
    E = np.random.default_rng(7).normal(size=(sx.shape[0], 16))
    rn, _ = LR.propose(kern, sx, sy, t, m, E, 16, 0.25, 1, 4096, rows=rows)
    assert LR.recall(sp, exact) > LR.recall(rn, exact)
