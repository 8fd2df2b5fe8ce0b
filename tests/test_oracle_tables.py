"""Pins for the oracle's physics tables: each closed form against an
independent quadrature of its differential form, textbook limits, and a
cut-derivative identity tying the restricted stopping powers to the Moller
and Bhabha differential cross sections."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import tables as T

PB = T.Material(82.0, 207.2, 11.35, 823.0)
LAR = T.Material(18.0, 39.948, 1.396, 188.0)
BARN = 1e-24


def quad(f, a, b, **kw):
    v, err = integrate.quad(f, a, b, epsabs=0.0, epsrel=1e-13, limit=400, **kw)
    return v


# ---------------------------------------------------------------- grid / materials
def test_grid():
    E = T.grid_energies()
    assert len(E) == 181
    assert E[0] == pytest.approx(1e-3, rel=1e-15)
    assert E[-1] == pytest.approx(1e6, rel=1e-13)
    assert np.allclose(np.diff(np.log(E)), math.log(10) / 20, rtol=1e-12)


def test_material_densities():
    # n_at = rho N_A / A ; radiation length from the PDG fit is within 2% of
    # the PDG tabulated 6.37 (Pb) and 19.55 (Ar) g/cm^2
    assert PB.n_at == pytest.approx(11.35 * 6.02214076e23 / 207.2, rel=1e-15)
    assert PB.n_el == pytest.approx(82 * PB.n_at, rel=1e-15)
    assert PB.X0_gcm2 == pytest.approx(6.37, rel=0.02)
    assert LAR.X0_gcm2 == pytest.approx(19.55, rel=0.02)


# ---------------------------------------------------------------- Compton
@pytest.mark.parametrize("E", [1e-3, 0.01, 0.1, 1.0, 10.0, 1e3, 1e5])
def test_klein_nishina_closed_form_equals_quadrature(E):
    k = E / T.ME
    e0 = 1.0 / (1.0 + 2.0 * k)
    # integrate in ln(eps) for accuracy at large k
    q = quad(lambda l: T.dsigma_klein_nishina_deps(E, math.exp(l)) * math.exp(l), math.log(e0), 0.0)
    assert T.sigma_klein_nishina(E) == pytest.approx(q, rel=1e-9)


def test_klein_nishina_thomson_limit():
    # low-energy series: sigma/sigma_T = 1 - 2k + 26/5 k^2 - 133/10 k^3 + 1144/35 k^4 + ...
    for k in (1e-3, 3e-3):
        series = 1 - 2 * k + 26 / 5 * k ** 2 - 133 / 10 * k ** 3 + 1144 / 35 * k ** 4
        assert T.sigma_klein_nishina(k * T.ME) / T.SIGMA_THOMSON == pytest.approx(series, rel=5e-9)
    assert T.SIGMA_THOMSON / BARN == pytest.approx(0.66524587, rel=1e-7)


# ---------------------------------------------------------------- photoelectric
def test_photoelectric_scaling():
    # Z^5 E^-7/2 scaling (the prefactor is pinned by the golden-rule test below)
    s1 = T.sigma_photoelectric(0.2, 82.0)
    assert T.sigma_photoelectric(0.4, 82.0) / s1 == pytest.approx(2 ** -3.5, rel=1e-14)
    assert T.sigma_photoelectric(0.2, 41.0) / s1 == pytest.approx(2 ** -5, rel=1e-14)
    born = 4 * math.sqrt(2) * T.ALPHA ** 4 * 82 ** 5 * T.SIGMA_THOMSON * (T.ME / 0.2) ** 3.5
    assert s1 == pytest.approx(1.25 * born, rel=1e-14)


# Independent constants for the golden-rule pin below (CODATA 2018), so that
# a wrong constant in the oracle does not cancel out.
_ALPHA = 1.0 / 137.035999084
_ME_MEV = 0.51099895000
_HBARC_MEV_CM = 197.3269804e-13


def _k_shell_born_golden_rule(omega, Z):
    """K-shell photo-absorption cross section [cm^2] of a hydrogen-like atom of
    charge Z at photon energy omega [MeV], from first principles:
    Fermi's golden rule in the dipole approximation,
        sigma = 4 pi^2 alpha / (m^2 omega) * sum_f |<f| eps.p |1s>|^2 delta(E_f - E_i - omega),
    with a plane-wave final electron (Born approximation) and the 1s state
    psi(r) = exp(-r/a) / sqrt(pi a^3), a = 1/(Z alpha m), two K electrons.
    Natural units (hbar = c = 1, energies in MeV).  The momentum-space
    wavefunction phi(p) = (4 pi / p) int r psi(r) sin(p r) dr and the angular
    integral of (eps.p_hat)^2 are both done by quadrature here: nothing of the
    Heitler closed form (prefactor, powers of alpha, Z or omega) is assumed."""
    m = _ME_MEV
    a = 1.0 / (Z * _ALPHA * m)
    binding = 0.5 * (Z * _ALPHA) ** 2 * m
    p = math.sqrt(2.0 * m * (omega - binding))        # final momentum, non-relativistic
    kappa = p * a
    radial = integrate.quad(lambda x: x * math.exp(-x), 0.0, np.inf, weight="sin", wvar=kappa)[0]
    phi = 4.0 * math.pi / p * a * a * radial / math.sqrt(math.pi * a ** 3)
    ang = 2.0 * math.pi * quad(lambda c: c * c, -1.0, 1.0)          # int (eps.p_hat)^2 dOmega
    # sum over final plane waves: int d^3p/(2pi)^3 delta(p^2/2m - (omega - B)) = m p / (2 pi)^3 dOmega
    per_electron = 4.0 * math.pi ** 2 * _ALPHA / (m * m * omega) * m * p / (2.0 * math.pi) ** 3 \
        * p * p * ang * phi * phi
    return 2.0 * per_electron * _HBARC_MEV_CM ** 2


@pytest.mark.parametrize("Z", [1.0, 3.0, 8.0])
def test_photoelectric_normalisation_from_the_golden_rule(Z):
    """The oracle's K-shell term (its cross section divided by the all-shell
    factor 5/4, which is this reading's stated convention) is the high-energy
    limit of the non-relativistic Born K-shell cross section computed from the
    golden rule.  At omega = 100 MeV the finite-energy corrections
    (1 + 1/(pa)^2)^-4 and the binding energy are below 4e-5 for Z <= 8, so the
    two agree to 2e-4: a wrong power of alpha or Z, a wrong energy exponent or
    a wrong numerical prefactor in the oracle fails by orders of magnitude."""
    for omega in (100.0, 300.0):
        exact = _k_shell_born_golden_rule(omega, Z)
        assert T.sigma_photoelectric(omega, Z) / 1.25 == pytest.approx(exact, rel=2e-4), omega
    # and the approach to the limit is the expected one: with x = 1/(pa)^2 =
    # B/omega (B the binding energy), the factor (1 + x)^-4 lowers the exact
    # value by 4x and the binding, through p^-5 = (2 m (omega - B))^-5/2,
    # raises it by 5x/2: at 1 MeV the exact value lies 3x/2 below the limit
    m = _ME_MEV
    x = (Z * _ALPHA * m) ** 2 / (2.0 * m * 1.0)
    ratio = _k_shell_born_golden_rule(1.0, Z) / (T.sigma_photoelectric(1.0, Z) / 1.25)
    assert 1.0 - ratio == pytest.approx(1.5 * x, rel=0.05)


# ---------------------------------------------------------------- pair
@pytest.mark.parametrize("E", [1.1, 1.5, 3.0, 10.0, 1e3, 1e5])
def test_pair_closed_form_equals_quadrature(E):
    a = T.ME / E
    q = quad(lambda x: 1.0 - 4.0 / 3.0 * x * (1 - x), a, 1 - a) / PB.X0_cm
    assert T.sigma_pair_macro(E, PB.X0_cm) == pytest.approx(q, rel=1e-11)


def test_pair_limits():
    assert T.sigma_pair_macro(2 * T.ME, PB.X0_cm) == 0.0
    assert T.sigma_pair_macro(1e9, PB.X0_cm) == pytest.approx(7.0 / 9.0 / PB.X0_cm, rel=1e-8)


# ---------------------------------------------------------------- bremsstrahlung
def _dsig_brems(E, k, X0):
    y = k / E
    return (4 / 3 - 4 / 3 * y + y * y) / (k * X0)


@pytest.mark.parametrize("Tk,Ec", [(0.5, 0.1), (10.0, 0.1), (1000.0, 0.1), (10.0, 1.0), (1e5, 0.1)])
def test_brems_closed_forms_equal_quadrature(Tk, Ec):
    E = Tk + T.ME
    X0 = PB.X0_cm
    q = quad(lambda l: _dsig_brems(E, math.exp(l), X0) * math.exp(l), math.log(Ec), math.log(Tk))
    assert T.sigma_brems_macro(Tk, Ec, X0) == pytest.approx(q, rel=1e-11)
    kr = min(Ec, Tk)
    qs = quad(lambda k: k * _dsig_brems(E, k, X0), 0.0, kr)
    assert T.srad_subcut(Tk, Ec, X0) == pytest.approx(qs, rel=1e-11)


def test_brems_radiative_loss_limit():
    # with the cut at T the whole spectrum is sub-cut: S_rad -> E/X0 (x 0.99949 at 1 GeV since y_max = T/E)
    s = T.srad_subcut(1000.0, 1000.0, PB.X0_cm)
    assert s / ((1000.0 + T.ME) / PB.X0_cm) == pytest.approx(0.99949, abs=1e-5)


# ---------------------------------------------------------------- Moller / Bhabha
@pytest.mark.parametrize("Tk,Ec", [(0.25, 0.1), (1.0, 0.1), (10.0, 1.0), (1000.0, 0.1), (1e5, 0.1)])
def test_moller_bhabha_closed_forms_equal_quadrature(Tk, Ec):
    xc = Ec / Tk
    qm = quad(lambda l: T.dsigma_moller_deps(Tk, math.exp(l)) * math.exp(l), math.log(xc), math.log(0.5))
    assert T.sigma_moller(Tk, Ec) == pytest.approx(qm, rel=1e-10)
    qb = quad(lambda l: T.dsigma_bhabha_deps(Tk, math.exp(l)) * math.exp(l), math.log(xc), 0.0)
    assert T.sigma_bhabha(Tk, Ec) == pytest.approx(qb, rel=1e-10)


def test_moller_bhabha_ultrarelativistic_limits():
    Tk = 1e7
    g, b2 = T._kin(Tk)
    pref = 2 * math.pi * T.RE ** 2 / (g - 1)
    for eps in (0.01, 0.2, 0.45):
        m = T.dsigma_moller_deps(Tk, eps) * b2 / pref
        assert m == pytest.approx(1 + 1 / eps ** 2 + 1 / (1 - eps) ** 2, rel=1e-6)
        b = T.dsigma_bhabha_deps(Tk, eps) / pref
        assert b == pytest.approx((1 - eps + eps * eps) ** 2 / eps ** 2, rel=1e-6)


def test_rejection_bounds():
    # Moller envelope 1 + C1/4 + max(0, 1 - C2) bounds eps^2 [bracket]; Bhabha acceptance <= 1
    for Tk in np.geomspace(0.21, 1e6, 60):
        g, b2 = T._kin(Tk)
        C1 = ((g - 1) / g) ** 2
        C2 = (2 * g - 1) / (g * g)
        bound = 1 + C1 / 4 + max(0.0, 1 - C2)
        eps = np.linspace(1e-6, 0.5, 2001)
        f = eps ** 2 * (C1 + 1 / eps ** 2 + 1 / (1 - eps) ** 2 - C2 / (eps * (1 - eps)))
        assert f.max() <= bound * (1 + 1e-12)
        B1, B2, B3, B4 = T.bhabha_B(Tk)
        e = np.linspace(1e-6, 1.0, 2001)
        acc = 1 - b2 * (B1 * e - B2 * e ** 2 + B3 * e ** 3 - B4 * e ** 4)
        assert acc.max() <= 1.0 + 1e-12 and acc.min() >= -1e-12


# ---------------------------------------------------------------- stopping power
@pytest.mark.parametrize("mat", [PB, LAR])
@pytest.mark.parametrize("Tk", [1.0, 10.0, 1000.0])
def test_restricted_loss_cut_derivative_identity(mat, Tk):
    # d S_col / d Ec = n_el Ec dsigma/dT_delta(Ec): moving the cut moves delta
    # rays of energy Ec between the continuous and the discrete part
    Ec, h = 0.1, 1e-5
    for positron, dsig in ((False, T.dsigma_moller_deps), (True, T.dsigma_bhabha_deps)):
        d = (T.scol_restricted(Tk, Ec + h, mat, positron) - T.scol_restricted(Tk, Ec - h, mat, positron)) / (2 * h)
        expect = mat.n_el * Ec * dsig(Tk, Ec / Tk) / Tk
        assert d == pytest.approx(expect, rel=2e-7)


def test_unrestricted_limits_rohrlich_carlson():
    # with the cut above the maximum transfer, the restricted forms reduce to
    # the Rohrlich-Carlson unrestricted stopping powers
    mat = PB
    for Tk in (0.01, 0.05, 0.09):
        g, b2 = T._kin(Tk)
        tau = Tk / T.ME
        Im = mat.I_eV * 1e-6 / T.ME
        dlt = T.density_effect(Tk, mat)
        pre = 2 * math.pi * T.RE ** 2 * T.ME * mat.n_el / b2
        lg = math.log(tau * tau * (tau + 2) / (2 * Im * Im))
        fm = 1 - b2 + (tau * tau / 8 - (2 * tau + 1) * math.log(2)) / (tau + 1) ** 2
        fp = 2 * math.log(2) - b2 / 12 * (23 + 14 / (tau + 2) + 10 / (tau + 2) ** 2 + 4 / (tau + 2) ** 3)
        assert T.scol_restricted(Tk, 1.0, mat, False) == pytest.approx(pre * (lg + fm - dlt), rel=1e-12)
        assert T.scol_restricted(Tk, 1.0, mat, True) == pytest.approx(pre * (lg + fp - dlt), rel=1e-12)


def test_density_effect_high_energy_asymptote():
    # 2 ln(hw_p/I) + 2 ln(beta gamma) - 1, clamped at zero at low energy
    assert T.density_effect(0.01, PB) == 0.0
    g, b2 = T._kin(1e4)
    hwp = 28.816 * math.sqrt(11.35 * 82 / 207.2)
    assert T.density_effect(1e4, PB) == pytest.approx(2 * math.log(hwp / 823) + 2 * math.log(math.sqrt(b2) * g) - 1,
                                                     rel=1e-14)


def test_stopping_power_positive_on_grid():
    for mat in (PB, LAR):
        for e in T.grid_energies():
            for pos in (False, True):
                assert T.stopping_power(e, 0.1, mat, pos) > 0.0


# ---------------------------------------------------------------- range
@pytest.mark.parametrize("positron", [False, True])
@pytest.mark.parametrize("mat", [PB, LAR])
def test_range_table_equals_independent_quadrature(positron, mat):
    Ec = 0.1
    R = T.range_table(Ec, mat, positron)
    E = T.grid_energies()
    S = lambda t: T.stopping_power(t, Ec, mat, positron)  # noqa: E731
    # kinks of S: the delta-ray cut switch (T = Ec or 2 Ec) and the density-effect onset
    onset = [t for t in E if T.density_effect(t, mat) > 0.0][0]
    kinks = [Ec, 2 * Ec, onset]
    # 1) interval increments, away from the kinks: 8-point Gauss-Legendre in ln T is exact to ~1e-13
    n_checked = 0
    for i in range(0, 180, 7):
        a, b = E[i], E[i + 1]
        if any(a / 1.2 <= k <= b * 1.2 for k in kinks):
            continue
        q = quad(lambda t: 1.0 / S(t), a, b)
        assert R[i + 1] - R[i] == pytest.approx(q, rel=1e-11), i
        n_checked += 1
    assert n_checked > 15
    # 2) cumulative value, including the kinked intervals (GL-8 error there ~1e-7)
    R0 = E[0] / S(E[0])
    assert R[0] == R0
    for i in (20, 80, 99, 140, 180):
        pts = sorted(k for k in kinks if E[0] < k < E[i])
        edges = [E[0]] + pts + [E[i]]
        q = R0 + sum(quad(lambda t: 1.0 / S(t), a, b) for a, b in zip(edges[:-1], edges[1:]))
        assert R[i] == pytest.approx(q, rel=1e-6), i
    assert np.all(np.diff(R) > 0)


def test_lookup_and_inverse_range_roundtrip():
    R = T.range_table(0.1, PB, False)
    for Tk in np.geomspace(0.1, 1e5, 200):
        assert T.inverse_range(R, T.lookup(R, Tk)) == pytest.approx(Tk, rel=1e-12)
    E = T.grid_energies()
    for i in (0, 17, 180):
        assert T.lookup(R, E[i]) == pytest.approx(R[i], rel=1e-12)
