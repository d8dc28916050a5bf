"""Pins for the oracle's correlation-based neighbor sets (CPU only).

* the lag-pruned search returns exactly the brute-force sets (Alg. 2 is an
  exact kNN among earlier points, so the plain definition is the reference);
* for the anisotropic Matern kernel the sets equal Euclidean nearest neighbors
  in scaled coordinates (the coordinate transformation the paper mentions for
  kernels that admit one), computed by SciPy's distance routine;
* for the Gneiting kernel the key order agrees with the order of the FP64
  correlation itself (no near-ties on these seeds);
* sets are invariant under exactly representable translations of space and time.
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import synth
from oracle import neighbors as NB
from oracle import kernels as K


def _small(kind, seed=0, n_sites=120, n_times=6, stations=None):
    d = synth.config_small(seed=seed, n_sites=n_sites, n_times=n_times, k=0, m=10, kind=kind,
                           n_stations=stations)
    return d


@pytest.mark.parametrize("kind", [1, 2, 3])
@pytest.mark.parametrize("m", [1, 7, 30])
def test_lag_pruned_equals_brute_force(kind, m):
    d = _small(kind)
    X = (d["sx"], d["sy"], d["t"])
    a = NB.brute_force(d["kern"], *X, m)
    b = NB.lag_pruned(d["kern"], *X, m)
    assert np.array_equal(a, b)


def test_lag_pruned_equals_brute_force_stations_with_missing_days():
    d = _small(1, stations=300, n_times=8)
    X = (d["sx"], d["sy"], d["t"])
    a = NB.brute_force(d["kern"], *X, 30)
    b = NB.lag_pruned(d["kern"], *X, 30)
    assert np.array_equal(a, b)


def test_padding_and_first_rows():
    d = _small(1)
    X = (d["sx"], d["sy"], d["t"])
    nb = NB.brute_force(d["kern"], *X, 10)
    assert (nb[0] == -1).all()
    for i in range(1, 10):
        assert sorted(nb[i, :i].tolist()) == list(range(i))
        assert (nb[i, i:] == -1).all()
    assert (nb[10:] >= 0).all()
    assert all(len(set(r)) == len(r) for r in nb[10:].tolist())
    assert (nb[np.arange(nb.shape[0])[:, None].repeat(10, 1) <= nb].size == 0)


def test_matern_aniso_equals_scaled_euclidean_knn():
    d = _small(3, n_sites=150, n_times=5)
    kern = d["kern"]
    sx, sy, t = d["sx"], d["sy"], d["t"]
    m = 10
    nb = NB.brute_force(kern, sx, sy, t, m)
    Y = np.stack([sx / kern["range_s"], sy / kern["range_s"], t / kern["range_t"]], 1)
    Dm = cdist(Y, Y)
    for i in range(1, sx.shape[0]):
        order = np.argsort(Dm[i, :i], kind="stable")[:m]
        assert np.array_equal(nb[i, :min(i, m)], order), i


def test_gneiting_key_order_equals_correlation_order():
    d = _small(1, n_sites=200, n_times=6)
    X = (d["sx"], d["sy"], d["t"])
    rows = np.arange(1, d["n"])
    nb = NB.brute_force(d["kern"], *X, 20)
    assert NB.rho_order_mismatches(d["kern"], *X, nb[1:], rows) == []
    # sets equal to a ranking by the exp-based correlation
    for i in rows[::7]:
        js = np.arange(i)
        rho = K.correlation(d["kern"], X[0][js] - X[0][i], X[1][js] - X[1][i], X[2][i] - X[2][js])
        order = np.lexsort((js, -rho))[:20]
        assert np.array_equal(nb[i, :min(i, 20)], order), i


def test_translation_invariance():
    d = _small(1, n_sites=150, n_times=6)
    q = 2.0 ** -30
    sx = np.round(d["sx"] / q) * q
    sy = np.round(d["sy"] / q) * q
    t = d["t"]
    a = NB.brute_force(d["kern"], sx, sy, t, 12)
    b = NB.brute_force(d["kern"], sx + 0.5, sy - 2.0, t + 7.0, 12)
    assert np.array_equal(a, b)


def test_ties_go_to_lower_index():
    # duplicated locations at the same time: equal keys
    sx = np.array([0.1, 0.1, 0.1, 0.5, 0.1])
    sy = np.array([0.2, 0.2, 0.2, 0.5, 0.2])
    t = np.zeros(5)
    kern = synth.kern_gneiting()
    nb = NB.brute_force(kern, sx, sy, t, 2)
    assert nb[4].tolist() == [0, 1]
    assert nb[3].tolist() == [0, 1]


def test_wrong_order_key_would_be_caught():
    """A plausible slip (dropping the temporal term of the key) changes the sets."""
    d = _small(1)
    X = (d["sx"], d["sy"], d["t"])
    good = NB.brute_force(d["kern"], *X, 10)
    bad_kern = dict(d["kern"], tau=0.0)
    bad = NB.brute_force(bad_kern, *X, 10)
    assert not np.array_equal(good, bad)
