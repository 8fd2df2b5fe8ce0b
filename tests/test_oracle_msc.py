"""Pins of the oracle's optional multiple-scattering deflection.

* Width: at a thickness of beta^2 X0 the logarithmic correction of the
  Highland width vanishes, so theta0 = 13.6 MeV / p exactly (p from the
  kinetic energy by relativistic kinematics); at fixed thickness theta0 * p is
  constant for ultra-relativistic particles; no deflection for s = 0 or below
  the point where the correction bracket reaches zero.
* Sampling: with u = +z the two projected angles are independent Gaussians
  of width theta0 (Kolmogorov-Smirnov against the normal law, zero
  correlation), so the mean squared space angle is 2 theta0^2.
* Geometry: deflected directions are unit vectors and the distribution of the
  deflection angle does not depend on the initial direction.
* Transport: the deflection changes no energy, so the per-event energy ledger
  stays exact with scattering on, and without it nothing changes.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads

ME = 0.51099895


def _kin(T):
    p = math.sqrt(T * (T + 2 * ME))
    return p, p / (T + ME)


@pytest.mark.parametrize("T", [0.3, 2.0, 50.0, 1000.0])
def test_width_at_thickness_beta2_X0_is_13_6_over_p(T):
    p, beta = _kin(T)
    X0 = 0.56
    assert oracle.msc_theta0(T, beta * beta * X0, X0) == pytest.approx(13.6 / p, rel=1e-12)


def test_width_times_momentum_constant_when_ultrarelativistic():
    X0, s = 14.0, 0.7
    v = [oracle.msc_theta0(T, s, X0) * _kin(T)[0] for T in (1e4, 3e4, 1e5)]
    assert max(v) / min(v) - 1 < 1e-7


def test_no_deflection_for_zero_or_vanishing_bracket():
    assert oracle.msc_theta0(10.0, 0.0, 1.0) == 0.0
    assert oracle.msc_theta0(10.0, 1e-13, 1.0) == 0.0       # x / beta^2 ~ 1e-13: bracket <= 0
    assert oracle.msc_theta0(10.0, 1e-9, 1.0) > 0.0


def _tracks(n, u, rng):
    t = np.zeros(n, dtype=oracle.TRACK_DTYPE)
    t["event"] = 7
    t["key"] = rng.integers(0, 2 ** 62, n)
    t["step"] = rng.integers(0, 50, n)
    t["type"] = 1
    t["alive"] = 1
    t["T"] = 100.0
    t["u"] = u
    return t


def _problem(msc=True):
    w = workloads.electron_showers_1gev_field(1)
    return oracle.problem_for(w, msc=msc), w


def test_projected_angles_are_gaussian_with_width_theta0():
    pb, w = _problem()
    rng = np.random.default_rng(5)
    n = 20000
    t = _tracks(n, (0.0, 0.0, 1.0), rng)
    T, s = 100.0, 0.05
    theta0 = oracle.msc_theta0(T, s, pb.x0_cm[0])
    assert 0.005 < theta0 < 0.05
    pb.msc_deflect(t, 0, T, s)
    u = t["u"]
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-14)
    tx = np.arctan2(u[:, 0], u[:, 2]) / theta0
    ty = np.arctan2(u[:, 1], u[:, 2]) / theta0
    for a in (tx, ty):
        assert stats.kstest(a, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(tx, ty)[0, 1]) < 4 / math.sqrt(n)
    th2 = np.arccos(np.clip(u[:, 2], -1, 1)) ** 2
    assert np.mean(th2) == pytest.approx(2 * theta0 ** 2, rel=4 * math.sqrt(2.0 / n) * 2)


def test_deflection_angle_independent_of_initial_direction():
    pb, w = _problem()
    rng = np.random.default_rng(9)
    n = 8000
    T, s = 5.0, 0.02
    a = _tracks(n, (0.0, 0.0, 1.0), rng)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    v[:10] = (0.0, 0.0, -1.0)                       # the pole branch of the rotation
    b = _tracks(n, v, rng)
    b["u"] = v
    u0 = b["u"].copy()
    pb.msc_deflect(a, 1, T, s)
    pb.msc_deflect(b, 1, T, s)
    ca = a["u"][:, 2]
    cb = np.sum(b["u"] * u0, axis=1)
    assert np.allclose(np.linalg.norm(b["u"], axis=1), 1.0, atol=1e-13)
    assert stats.ks_2samp(ca, cb).pvalue > 1e-3


def test_showers_with_scattering_conserve_energy_and_off_changes_nothing():
    w = workloads.electron_showers_1gev_field(6, n_slots=1 << 12)
    tr, rows = oracle.tracks_from_primaries(w.primaries)
    e_on, l_on, st_on = oracle.problem_for(w, msc=True).run_events(tr, rows, w.n_events, 4)
    e_off, l_off, st_off = oracle.problem_for(w, msc=False).run_events(tr, rows, w.n_events, 4)
    e_def, l_def, st_def = oracle.problem_for(w).run_events(tr, rows, w.n_events, 4)
    assert st_off == st_def and np.array_equal(e_off, e_def)
    assert st_on != st_off                         # scattering changes the histories
    T0 = w.primaries["T"]
    for e, l in ((e_on, l_on), (e_off, l_off)):
        tot = e.sum(1) + l["escaped"] + 2 * ME * (l["n_pair"].astype(float) - l["n_annih"])
        assert np.max(np.abs(tot - T0) / T0) < 1e-9
