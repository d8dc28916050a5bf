"""Pins for the oracle's correlation-based neighbor sets (CPU only).

* the lag-pruned search returns exactly the brute-force sets (Alg. 2 is an
  exact kNN among earlier points, so the plain definition is the reference);
* for the anisotropic Matern kernel the sets equal Euclidean nearest neighbors
  in scaled coordinates (the coordinate transformation the paper mentions for
  kernels that admit one), computed by SciPy's distance routine;
* for the Gneiting kernel the key order agrees with the order of the FP64
  correlation itself (no near-ties on these seeds);
* sets are invariant under exactly representable translations of space and time;
* every kernel setting the search supports -- Gneiting with gamma = 1/2 (sqrt)
  and gamma != 1/2 (pow), Gneiting-Matern at nu = 1/2, 3/2, 5/2 (log1p forms,
  checked against the Bessel-function correlation), anisotropic Matern -- ranks
  like its correlation, at integer and at real-valued times;
* real-valued times: the per-distinct-lag factors equal the integer-lag table
  where both apply, and the anisotropic sets equal scaled Euclidean kNN.
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


KERNELS = {
    "gneiting_sqrt": synth.kern_gneiting(),
    "gneiting_g035": synth.kern_gneiting(gamma=0.35),
    "gneiting_g045_b07": synth.kern_gneiting(gamma=0.45, beta=0.7, alpha=0.6),
    "gm_nu05": synth.kern_gneiting_matern(nu=0.5),
    "gm_nu15": synth.kern_gneiting_matern(nu=1.5),
    "gm_nu25": synth.kern_gneiting_matern(nu=2.5),
    "aniso_nu15": synth.kern_matern_aniso(),
}


def _real_times(t_int, rng, every_point=False):
    """Real-valued, nondecreasing times: integer time points moved to random real
    values (points of one time point keep a common time), or, with every_point,
    one distinct time per point."""
    if every_point:
        return np.sort(rng.uniform(0.0, float(t_int[-1]) + 1.0, t_int.shape[0]))
    vals = np.cumsum(rng.uniform(0.3, 1.7, int(t_int[-1]) + 1))
    return vals[t_int.astype(np.int64)]


@pytest.mark.parametrize("name", list(KERNELS))
@pytest.mark.parametrize("times", ["integer", "real", "real_every_point"])
def test_key_order_equals_correlation_order_all_kernels(name, times):
    """Sets and their order equal a ranking by the FP64 correlation itself
    (Gneiting-Matern through the Bessel-function form, which shares no code with
    the closed forms behind the key)."""
    kern = KERNELS[name]
    rng = np.random.default_rng(5)
    sx, sy, t = synth.grid_sites_times(90, 5, rng)
    sx, sy, t = synth.time_stratified_order(sx, sy, t, rng)
    if times != "integer":
        t = _real_times(t, rng, every_point=times == "real_every_point")
    X = (sx, sy, t)
    m = 15
    nb = NB.brute_force(kern, *X, m)
    rows = np.arange(1, sx.shape[0])
    assert NB.rho_order_mismatches(kern, *X, nb[1:], rows) == []
    bessel = kern["kind"] != 1
    for i in rows[::5]:
        js = np.arange(i)
        rho = K.correlation(kern, sx[js] - sx[i], sy[js] - sy[i], t[i] - t[js], bessel=bessel)
        order = np.lexsort((js, -rho))[:m]
        assert np.array_equal(nb[i, :min(i, m)], order), (name, times, i)


@pytest.mark.parametrize("name", list(KERNELS))
def test_general_lag_factors_equal_integer_table(name):
    kern = KERNELS[name]
    d = _small(1, seed=3, n_sites=80, n_times=5)
    X = (d["sx"], d["sy"], d["t"])
    a = NB.brute_force(kern, *X, 12)
    b = NB.brute_force(kern, *X, 12, general=True)
    assert np.array_equal(a, b)
    tab1, tab2 = NB.lag_tables(kern, 4)
    for lag in range(5):
        assert NB.lag_factors(kern, float(lag)) == (tab1[lag], tab2[lag])


def test_real_times_aniso_equals_scaled_euclidean_knn():
    kern = KERNELS["aniso_nu15"]
    rng = np.random.default_rng(8)
    sx, sy, t = synth.grid_sites_times(100, 6, rng)
    sx, sy, t = synth.time_stratified_order(sx, sy, t, rng)
    t = _real_times(t, rng)
    m = 10
    nb = NB.brute_force(kern, sx, sy, t, m)
    Y = np.stack([sx / kern["range_s"], sy / kern["range_s"], t / kern["range_t"]], 1)
    Dm = cdist(Y, Y)
    for i in range(1, sx.shape[0]):
        order = np.argsort(Dm[i, :i], kind="stable")[:m]
        assert np.array_equal(nb[i, :min(i, m)], order), i


def test_real_times_translation_invariance():
    """Times on a 2^-20 grid, shifted by an exactly representable 0.25: every lag
    t_i - t_j is unchanged bit for bit, so the sets are too."""
    rng = np.random.default_rng(9)
    sx, sy, t = synth.grid_sites_times(80, 5, rng)
    sx, sy, t = synth.time_stratified_order(sx, sy, t, rng)
    q = 2.0 ** -20
    t = np.round(_real_times(t, rng) / q) * q
    for kern in (KERNELS["gneiting_g035"], KERNELS["gm_nu25"]):
        a = NB.brute_force(kern, sx, sy, t, 9)
        b = NB.brute_force(kern, sx, sy, t + 0.25, 9)
        assert np.array_equal(a, b)


def test_real_times_floor_of_lag_would_be_caught():
    """A plausible slip for real times -- taking the factors at the integer part
    of the lag -- changes the sets."""
    kern = KERNELS["gneiting_sqrt"]
    rng = np.random.default_rng(10)
    sx, sy, t = synth.grid_sites_times(80, 6, rng)
    sx, sy, t = synth.time_stratified_order(sx, sy, t, rng)
    t = _real_times(t, rng)
    good = NB.brute_force(kern, sx, sy, t, 10)
    tabs = NB.lag_tables(kern, int(np.ceil(t[-1] - t[0])) + 1)
    bad = np.full_like(good, -1)
    for i in range(1, sx.shape[0]):
        js = np.arange(i)
        tau = np.floor(t[i] - t[js]).astype(np.int64)
        kk = -(tabs[0][tau] + np.sqrt((sx[js] - sx[i]) ** 2 + (sy[js] - sy[i]) ** 2) * tabs[1][tau])
        sel = js[np.lexsort((js, -kk))[:10]]
        bad[i, :sel.shape[0]] = sel
    assert not np.array_equal(good, bad)


def test_lag_pruned_refuses_real_times():
    rng = np.random.default_rng(11)
    sx, sy, t = synth.grid_sites_times(20, 3, rng)
    with pytest.raises(ValueError):
        NB.lag_pruned(KERNELS["gneiting_sqrt"], sx, sy, t + 0.5 * (t > 0), 5)
