"""Pins for the oracle's covariance kernels (CPU only).

* closed forms for nu in {1/2, 3/2, 5/2} against the Bessel definition
  2^(1-nu)/Gamma(nu) x^nu K_nu(x) (SciPy), Eq. (Gneiting);
* effective ranges printed in the paper's parameter tables (golden fixture),
  with the printing precision of each parameter propagated to the range;
* zero time lag reduces Eq. (Gneiting) to an isotropic Matern, gamma = 0 makes
  it separable (both stated right after Eq. (Gneiting));
* the stretched-exponential Gneiting form equals Eq. (Gneiting) at nu = 1/2.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import kernels as K

GOLD = os.path.join(os.path.dirname(__file__), "golden", "effective_ranges.json")


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_closed_forms_match_bessel(nu):
    x = np.concatenate([np.linspace(1e-6, 1.0, 200), np.linspace(1.0, 40.0, 400)])
    a = K.matern_closed(nu, x)
    b = K.matern_bessel(nu, x)
    assert np.max(np.abs(a - b) / np.maximum(b, 1e-300)) < 1e-12


def _row_kern(r):
    return {"kind": K.GNEITING_MATERN, "sigma2": 1.0, "a": r["a"], "c": r["c"], "alpha": r["alpha"],
            "gamma": r["gamma"], "delta": r["delta"], "nu": r["nu"]}


def _ranges(r, **over):
    kern = _row_kern(r)
    kern.update(over)
    return K.effective_ranges(kern, 0.05, bessel=(r["nu"] not in (0.5, 1.5, 2.5)))


def _propagated(r, half):
    """Linearised effect of printing precision on (time, space) ranges."""
    base = np.array(_ranges(r))
    tot = np.zeros(2)
    for p in ("a", "c", "alpha", "gamma", "delta"):
        h = half[p]
        if h == 0:
            continue
        up = np.array(_ranges(r, **{p: r[p] + h}))
        dn = np.array(_ranges(r, **{p: r[p] - h}))
        with np.errstate(invalid="ignore"):
            tot += np.nan_to_num(np.maximum(np.abs(up - base), np.abs(dn - base)), posinf=0.0)
    return tot


def _gold():
    with open(GOLD) as f:
        return json.load(f)


def _ids(rows):
    return [f'{r["table"]}-{r["date"]}' for r in rows]


G = _gold()


@pytest.mark.parametrize("row", G["rows"], ids=_ids(G["rows"]))
def test_effective_time_range(row):
    half = G["printing"][row["table"]]
    tr, _ = _ranges(row)
    if row["time"] == "inf":
        assert tr > 1e6
        return
    tol = _propagated(row, half)[0] + half["time"] + 1e-9
    key = f'{row["table"]} {row["date"]} time'
    if key in G["known_inconsistent"]:
        assert abs(tr - row["time"]) > tol, "row listed as inconsistent now reproduces; update the fixture"
        pytest.xfail(G["known_inconsistent"][key])
    assert abs(tr - row["time"]) <= tol, (tr, row["time"], tol)


@pytest.mark.parametrize("row", G["rows"], ids=_ids(G["rows"]))
def test_effective_space_range(row):
    half = G["printing"][row["table"]]
    _, sr = _ranges(row)
    key = f'{row["table"]} {row["date"]} space'
    if "space_km" in row:
        got, want = sr / 1000.0, row["space_km"]
        tol = _propagated(row, half)[1] / 1000.0 + half["space"]
    else:
        got, want = sr, row["space"]
        tol = _propagated(row, half)[1] + half["space"]
    if key in G["known_inconsistent"]:
        assert abs(got - want) > tol, "row listed as inconsistent now reproduces; update the fixture"
        pytest.xfail(G["known_inconsistent"][key])
    assert abs(got - want) <= tol + 1e-9, (got, want, tol)


def test_zero_lag_is_matern():
    rng = np.random.default_rng(3)
    for nu in (0.5, 1.5, 2.5):
        kern = {"kind": K.GNEITING_MATERN, "sigma2": 1.7, "a": 0.3, "c": 4.0, "alpha": 0.7,
                "gamma": 0.6, "delta": 0.4, "nu": nu}
        h = rng.uniform(0, 2, 100)
        ang = rng.uniform(0, 2 * math.pi, 100)
        got = K.cov(kern, h * np.cos(ang), h * np.sin(ang), 0.0)
        want = 1.7 * K.matern_bessel(nu, 4.0 * h)
        assert np.allclose(got, want, rtol=1e-12, atol=0)


def test_gamma_zero_is_separable():
    rng = np.random.default_rng(4)
    kern = {"kind": K.GNEITING_MATERN, "sigma2": 2.0, "a": 0.8, "c": 3.0, "alpha": 0.5,
            "gamma": 0.0, "delta": 0.7, "nu": 1.5}
    dx, dy, dt = rng.normal(size=(3, 200))
    joint = K.cov(kern, dx, dy, dt) * K.cov(kern, 0.0, 0.0, 0.0)
    sep = K.cov(kern, dx, dy, 0.0) * K.cov(kern, 0.0, 0.0, dt)
    assert np.allclose(joint, sep, rtol=1e-13)
    kern["gamma"] = 0.5
    joint = K.cov(kern, dx, dy, dt) * K.cov(kern, 0.0, 0.0, 0.0)
    sep = K.cov(kern, dx, dy, 0.0) * K.cov(kern, 0.0, 0.0, dt)
    assert not np.allclose(joint, sep, rtol=1e-3)


def test_stretched_form_equals_paper_form_at_nu_half():
    rng = np.random.default_rng(5)
    for _ in range(20):
        a, c, alpha, beta, tau = rng.uniform(0.1, 2), rng.uniform(1, 30), rng.uniform(0.1, 1), \
            rng.uniform(0, 1), rng.uniform(1, 2)
        bj = {"kind": K.GNEITING, "sigma2": 1.3, "a": a, "c": c, "alpha": alpha, "beta": beta,
              "gamma": 0.5, "tau": tau}
        pg = 2 * beta * 0.5
        paper = {"kind": K.GNEITING_MATERN, "sigma2": 1.3, "a": a, "c": c, "alpha": alpha,
                 "gamma": pg, "delta": tau - pg, "nu": 0.5}
        dx, dy = rng.normal(scale=0.2, size=(2, 50))
        dt = rng.integers(0, 20, 50).astype(float)
        assert np.allclose(K.cov(bj, dx, dy, dt), K.cov(paper, dx, dy, dt), rtol=1e-13, atol=0)


def test_matern_aniso_is_matern_of_scaled_distance():
    kern = {"kind": K.MATERN_ANISO, "sigma2": 1.0, "range_s": 0.2, "range_t": 3.0, "nu": 1.5}
    rng = np.random.default_rng(6)
    dx, dy, dt = rng.normal(size=(3, 100))
    d = np.sqrt((dx / 0.2) ** 2 + (dy / 0.2) ** 2 + (dt / 3.0) ** 2)
    assert np.allclose(K.cov(kern, dx, dy, dt), K.matern_bessel(1.5, d), rtol=1e-12)
