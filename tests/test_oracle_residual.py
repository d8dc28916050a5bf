"""Pins for the oracle's residual-correlation neighbor sets (CPU only).

* without inducing points the residual is the covariance itself, so the sets
  equal the correlation-based sets of the plain search (a separate oracle,
  pinned on its own);
* the residual covariance equals the conditional covariance of the latent
  process given its values at the inducing points, computed here by Gaussian
  conditioning through the inverse of the joint covariance matrix (a different
  route from the oracle's Cholesky and triangular solve), and the ranking by
  |r_ij| / sqrt(r_ii r_jj) of that matrix gives the oracle's sets; residual
  correlations of both signs occur, so a dropped absolute value shows;
* a data point that coincides with an inducing point has no residual variance
  and is never chosen while other candidates remain;
* the sets do not change when sigma2 is scaled (correlations are scale free);
* equal keys go to the lower index.
"""
import numpy as np
import pytest

import synth
from oracle import kernels as K
from oracle import neighbors as NB
from oracle import residual as RS


def _problem(seed=0, n_sites=40, n_times=4, k=10, kind=1):
    d = synth.config_small(seed=seed, n_sites=n_sites, n_times=n_times, k=k, m=8, kind=kind)
    X = (d["sx"], d["sy"], d["t"])
    Z = (d["zx"], d["zy"], d["zt"]) if k else None
    return d, X, Z


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_no_inducing_points_equals_correlation_search(kind):
    d, X, _ = _problem(kind=kind, k=0)
    for m in (1, 6, 20):
        assert np.array_equal(RS.brute_force(d["kern"], X, None, m), NB.brute_force(d["kern"], *X, m))


def _conditional_cov(kern, X, Z):
    """C_XX - C_XZ C_ZZ^-1 C_ZX as the inverse of the X block of the joint precision."""
    P = (np.concatenate([Z[0], X[0]]), np.concatenate([Z[1], X[1]]), np.concatenate([Z[2], X[2]]))
    J = K.cov_matrix(kern, P, P)
    k = Z[0].shape[0]
    Q = np.linalg.inv(J)
    return np.linalg.inv(Q[k:, k:])


def test_residual_equals_gaussian_conditioning():
    # A rough (exponential) kernel keeps the joint covariance well conditioned;
    # inducing points drawn apart from the data (kMeans centres of one-point
    # clusters would coincide with data points, whose residual is then zero).
    d, X, _ = _problem(seed=3, n_sites=30, n_times=3, k=0, kind=2)
    rng = np.random.default_rng(3)
    Z = (rng.uniform(0, 1, 8), rng.uniform(0, 1, 8), rng.uniform(0, 2, 8))
    kern = dict(d["kern"], nu=0.5, c=5.0, a=2.0)
    R = _conditional_cov(kern, X, Z)
    U, dv = RS.residual_parts(kern, X, Z)
    n = X[0].shape[0]
    assert np.allclose(dv, np.diag(R), rtol=1e-7, atol=1e-10)
    for i in (5, 17, n // 2, n - 1):
        js = np.arange(i)
        c = K.cov(kern, X[0][i] - X[0][js], X[1][i] - X[1][js], X[2][i] - X[2][js])
        assert np.allclose(c - U[js] @ U[i], R[i, js], rtol=1e-7, atol=1e-10)
    assert (R[np.tril_indices(n, -1)] < 0).any() and (R[np.tril_indices(n, -1)] > 0).any()
    m = 7
    want = np.full((n, m), -1, dtype=np.int32)
    for i in range(1, n):
        js = np.arange(i)
        rho = np.abs(R[i, js]) / np.sqrt(R[i, i] * np.diag(R)[js])
        order = np.lexsort((js, -rho))[:m]
        want[i, :order.shape[0]] = js[order]
    assert np.array_equal(RS.brute_force(kern, X, Z, m), want)


def test_point_at_an_inducing_point_is_not_chosen():
    d, X, Z = _problem(seed=5, k=10)
    j = 7
    Z = (Z[0].copy(), Z[1].copy(), Z[2].copy())
    Z[0][0], Z[1][0], Z[2][0] = X[0][j], X[1][j], X[2][j]
    U, dv = RS.residual_parts(d["kern"], X, Z)
    assert abs(dv[j]) < 1e-10
    nb = RS.brute_force(d["kern"], X, Z, 8)
    for i in range(j + 9, X[0].shape[0]):
        assert j not in nb[i]


def test_scale_invariance():
    d, X, Z = _problem(seed=6, k=12)
    a = RS.brute_force(d["kern"], X, Z, 9)
    b = RS.brute_force(dict(d["kern"], sigma2=3.0 * d["kern"]["sigma2"]), X, Z, 9)
    assert np.array_equal(a, b)


def test_ties_go_to_lower_index():
    d, X, Z = _problem(seed=7, k=6)
    sx, sy, t = (a.copy() for a in X)
    # two later points at the same place and time as point 3: equal keys for every query
    sx[[4, 5]], sy[[4, 5]], t[[4, 5]] = sx[3], sy[3], t[3]
    X2 = (sx, sy, t)
    nb = RS.brute_force(d["kern"], X2, Z, 12)
    for i in range(6, 40):
        row = list(nb[i])
        pos = [row.index(q) for q in (3, 4, 5) if q in row]
        assert pos == sorted(pos)
