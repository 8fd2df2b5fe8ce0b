"""Oracle physics tables for the EM shower step loop -- TEST INFRASTRUCTURE ONLY.

This module is part of the oracle: a plain, slow, FP64 definition of what the
device path must compute.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it; the product path
(``paper_2503_17608_amd``) never does, and builds its own tables on the device.

The paper (arXiv 2503.17608) gives no physics formulas: it says only that the
transport covers electromagnetic processes for photons, electrons and
positrons (Introduction; Stepping algorithm).  The processes and the formulas
below are the reading this project takes of that statement, each a named
textbook form:

* Klein-Nishina total cross section per electron (Compton);
* Born K-shell photoelectric cross section (Heitler) scaled by 5/4 for all shells;
* Bethe-Heitler pair production with complete screening (Tsai / PDG), macroscopic;
* Moller and Bhabha cross sections above the production cut;
* Tsai complete-screening bremsstrahlung above the cut, and its sub-cut
  radiative loss;
* Berger-Seltzer restricted collision stopping power with a clamped
  high-energy density-effect correction;
* CSDA range by Gauss-Legendre quadrature of 1/S on the table grid.

Every table is sampled on a log-uniform kinetic-energy grid (1 keV .. 1 TeV,
20 nodes per decade, 181 nodes) and interpolated linearly in ln E.

Units: MeV, cm, g/cm^3, eV (mean excitation energy only).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# --- physical constants (CODATA 2018) -------------------------------------------
ME = 0.51099895            # electron rest energy [MeV]
RE = 2.8179403262e-13      # classical electron radius [cm]
ALPHA = 1.0 / 137.035999084
NA = 6.02214076e23         # Avogadro [1/mol]
HBAR_OMEGA_P_EV = 28.816   # plasma energy coefficient: 28.816 sqrt(rho Z/A) eV
SIGMA_THOMSON = 8.0 * math.pi * RE * RE / 3.0

# --- table grid ------------------------------------------------------------------
E_MIN = 1.0e-3             # MeV
N_PER_DECADE = 20
N_DECADES = 9
N_NODES = N_DECADES * N_PER_DECADE + 1   # 181

# table indices (per material); same order as the device library's table blob
T_COMPTON, T_PHOTO, T_PAIR, T_MOLLER, T_BHABHA, T_BREMS, T_RANGE_EM, T_RANGE_EP = range(8)
N_TABLES = 8

# range step-limit parameters (final-range / fraction scheme)
RHO_RANGE = 0.2
R_FINAL = 0.01             # cm


@dataclass(frozen=True)
class Material:
    Z: float
    A: float        # g/mol
    rho: float      # g/cm^3
    I_eV: float     # mean excitation energy

    @property
    def n_at(self) -> float:
        return self.rho * NA / self.A

    @property
    def n_el(self) -> float:
        return self.Z * self.n_at

    @property
    def X0_gcm2(self) -> float:
        """Radiation length, PDG fit (Dahl): 716.4 A / (Z(Z+1) ln(287/sqrt Z))."""
        Z = self.Z
        return 716.4 * self.A / (Z * (Z + 1.0) * math.log(287.0 / math.sqrt(Z)))

    @property
    def X0_cm(self) -> float:
        return self.X0_gcm2 / self.rho


def grid_log_e0() -> float:
    return math.log(E_MIN)


def grid_dlog() -> float:
    return math.log(10.0) / N_PER_DECADE


def grid_energies() -> np.ndarray:
    """Node kinetic energies E_i = exp(ln E_min + i * ln(10)/20)."""
    l0, d = grid_log_e0(), grid_dlog()
    return np.array([math.exp(l0 + i * d) for i in range(N_NODES)])


# --- photons ---------------------------------------------------------------------
def sigma_klein_nishina(E: float) -> float:
    """Klein-Nishina total cross section per free electron [cm^2]."""
    k = E / ME
    l = math.log(1.0 + 2.0 * k)
    a = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k)
    b = l / (2.0 * k)
    c = (1.0 + 3.0 * k) / ((1.0 + 2.0 * k) ** 2)
    return 2.0 * math.pi * RE * RE * (a + b - c)


def dsigma_klein_nishina_deps(E: float, eps: float) -> float:
    """Klein-Nishina dsigma/deps per electron, eps = E'/E in [1/(1+2k), 1]."""
    k = E / ME
    one_minus_cos = (1.0 - eps) / (k * eps)
    sin2 = one_minus_cos * (2.0 - one_minus_cos)
    return math.pi * RE * RE / k * (1.0 / eps + eps - sin2)


def sigma_photoelectric(E: float, Z: float) -> float:
    """Born K-shell photoelectric cross section x 5/4 per atom [cm^2]."""
    return 1.25 * 4.0 * math.sqrt(2.0) * ALPHA ** 4 * Z ** 5 * SIGMA_THOMSON * (ME / E) ** 3.5


def pair_J(a: float) -> float:
    """Integral of x(1-x) over [a, 1-a]."""
    return (1.0 - 2.0 * a) / 2.0 - (1.0 - 3.0 * a + 3.0 * a * a - 2.0 * a ** 3) / 3.0


def sigma_pair_macro(E: float, X0_cm: float) -> float:
    """Complete-screening Bethe-Heitler pair cross section, macroscopic [1/cm]."""
    if E <= 2.0 * ME:
        return 0.0
    a = ME / E
    return ((1.0 - 2.0 * a) - 4.0 / 3.0 * pair_J(a)) / X0_cm


# --- electrons / positrons: delta rays ----------------------------------------------
def _kin(T: float):
    g = (T + ME) / ME
    b2 = 1.0 - 1.0 / (g * g)
    return g, b2


def sigma_moller(T: float, Ec: float) -> float:
    """Moller cross section per electron for delta rays above Ec [cm^2]; 0 if T <= 2 Ec."""
    if T <= 2.0 * Ec:
        return 0.0
    g, b2 = _kin(T)
    xc = Ec / T
    C1 = ((g - 1.0) / g) ** 2
    C2 = (2.0 * g - 1.0) / (g * g)
    br = C1 * (0.5 - xc) + 1.0 / xc - 1.0 / (1.0 - xc) - C2 * math.log((1.0 - xc) / xc)
    return 2.0 * math.pi * RE * RE / (b2 * (g - 1.0)) * br


def dsigma_moller_deps(T: float, eps: float) -> float:
    g, b2 = _kin(T)
    C1 = ((g - 1.0) / g) ** 2
    C2 = (2.0 * g - 1.0) / (g * g)
    return 2.0 * math.pi * RE * RE / (b2 * (g - 1.0)) * (
        C1 + 1.0 / eps ** 2 + 1.0 / (1.0 - eps) ** 2 - C2 / (eps * (1.0 - eps)))


def bhabha_B(T: float):
    g, _ = _kin(T)
    y = 1.0 / (1.0 + g)
    B1 = 2.0 - y * y
    B2 = (1.0 - 2.0 * y) * (3.0 + y * y)
    B4 = (1.0 - 2.0 * y) ** 3
    B3 = B4 + (1.0 - 2.0 * y) ** 2
    return B1, B2, B3, B4


def sigma_bhabha(T: float, Ec: float) -> float:
    """Bhabha cross section per electron for delta rays above Ec [cm^2]; 0 if T <= Ec."""
    if T <= Ec:
        return 0.0
    g, b2 = _kin(T)
    xc = Ec / T
    B1, B2, B3, B4 = bhabha_B(T)
    br = ((1.0 / xc - 1.0) / b2 - B1 * math.log(1.0 / xc) + B2 * (1.0 - xc)
          - B3 * (1.0 - xc * xc) / 2.0 + B4 * (1.0 - xc ** 3) / 3.0)
    return 2.0 * math.pi * RE * RE / (g - 1.0) * br


def dsigma_bhabha_deps(T: float, eps: float) -> float:
    g, b2 = _kin(T)
    B1, B2, B3, B4 = bhabha_B(T)
    return 2.0 * math.pi * RE * RE / (g - 1.0) * (
        1.0 / (b2 * eps * eps) - B1 / eps + B2 - B3 * eps + B4 * eps * eps)


# --- bremsstrahlung -----------------------------------------------------------------
def sigma_brems_macro(T: float, Ec: float, X0_cm: float) -> float:
    """Tsai complete-screening bremsstrahlung for photons above Ec [1/cm]; 0 if T <= Ec."""
    if T <= Ec:
        return 0.0
    E = T + ME
    yc, ym = Ec / E, T / E
    return (4.0 / 3.0 * math.log(ym / yc) - 4.0 / 3.0 * (ym - yc) + (ym * ym - yc * yc) / 2.0) / X0_cm


def srad_subcut(T: float, Ec: float, X0_cm: float) -> float:
    """Radiative stopping power from photons below min(Ec, T) [MeV/cm]."""
    E = T + ME
    yr = min(Ec, T) / E
    return E / X0_cm * (4.0 / 3.0 * yr - 2.0 / 3.0 * yr * yr + yr ** 3 / 3.0)


# --- restricted collision stopping power ----------------------------------------------
def density_effect(T: float, mat: Material) -> float:
    g, b2 = _kin(T)
    bg = math.sqrt(b2) * g
    hwp = HBAR_OMEGA_P_EV * math.sqrt(mat.rho * mat.Z / mat.A)
    return max(0.0, 2.0 * math.log(hwp / mat.I_eV) + 2.0 * math.log(bg) - 1.0)


def scol_restricted(T: float, Ec: float, mat: Material, positron: bool) -> float:
    """Berger-Seltzer restricted collision stopping power [MeV/cm]."""
    g, b2 = _kin(T)
    tau = T / ME
    Im = mat.I_eV * 1.0e-6 / ME
    if positron:
        D = min(Ec, T) / ME
        y = 1.0 / (g + 1.0)
        F = math.log(tau * D) - b2 / tau * (
            tau + 2.0 * D - 1.5 * D * D * y - (D - D ** 3 / 3.0) * y * y
            - (D * D / 2.0 - tau * D ** 3 / 3.0 + D ** 4 / 4.0) * y ** 3)
    else:
        D = min(Ec, T / 2.0) / ME
        F = (-1.0 - b2 + math.log((tau - D) * D) + tau / (tau - D)
             + (D * D / 2.0 + (2.0 * tau + 1.0) * math.log(1.0 - D / tau)) / (g * g))
    L = math.log(2.0 * (tau + 2.0) / (Im * Im)) + F - density_effect(T, mat)
    return 2.0 * math.pi * RE * RE * ME * mat.n_el / b2 * L


def stopping_power(T: float, Ec: float, mat: Material, positron: bool) -> float:
    """Total restricted stopping power S = S_col + S_rad (sub-cut) [MeV/cm]."""
    return scol_restricted(T, Ec, mat, positron) + srad_subcut(T, Ec, mat.X0_cm)


# Gauss-Legendre 8-point rule on [-1, 1] (library primitive)
_GL_X, _GL_W = np.polynomial.legendre.leggauss(8)


def range_table(Ec: float, mat: Material, positron: bool) -> np.ndarray:
    """CSDA range R(E_i): R_0 = E_0/S(E_0); each grid interval integrated
    with 8-point Gauss-Legendre in u = ln T of T/S(T)."""
    l0, d = grid_log_e0(), grid_dlog()
    E = grid_energies()
    R = np.empty(N_NODES)
    R[0] = E[0] / stopping_power(E[0], Ec, mat, positron)
    for i in range(N_NODES - 1):
        ua = l0 + i * d
        half = 0.5 * d
        mid = ua + half
        acc = 0.0
        for xk, wk in zip(_GL_X, _GL_W):
            t = math.exp(mid + half * xk)
            acc += wk * t / stopping_power(t, Ec, mat, positron)
        R[i + 1] = R[i] + half * acc
    return R


def build_tables(materials: list[Material], Ec: float) -> np.ndarray:
    """Table blob [n_materials, 8, 181] in FP64 (macroscopic 1/cm, range in cm)."""
    E = grid_energies()
    out = np.zeros((len(materials), N_TABLES, N_NODES))
    for m, mat in enumerate(materials):
        for i, e in enumerate(E):
            out[m, T_COMPTON, i] = mat.n_el * sigma_klein_nishina(e)
            out[m, T_PHOTO, i] = mat.n_at * sigma_photoelectric(e, mat.Z)
            out[m, T_PAIR, i] = sigma_pair_macro(e, mat.X0_cm)
            out[m, T_MOLLER, i] = mat.n_el * sigma_moller(e, Ec)
            out[m, T_BHABHA, i] = mat.n_el * sigma_bhabha(e, Ec)
            out[m, T_BREMS, i] = sigma_brems_macro(e, Ec, mat.X0_cm)
        out[m, T_RANGE_EM] = range_table(Ec, mat, positron=False)
        out[m, T_RANGE_EP] = range_table(Ec, mat, positron=True)
    return out


# --- table lookup (interpolation rule shared by both transport implementations) -----
def lookup(tab: np.ndarray, T: float) -> float:
    """Linear interpolation in ln T: t = (ln T - ln E0)/d, i = clamp(floor t, 0, N-2)."""
    t = (math.log(T) - grid_log_e0()) / grid_dlog()
    i = min(max(int(math.floor(t)), 0), N_NODES - 2)
    return tab[i] + (t - i) * (tab[i + 1] - tab[i])


def inverse_range(R: np.ndarray, r: float) -> float:
    """Exact inverse of the piecewise-linear forward range map."""
    j = int(np.searchsorted(R, r, side="right"))   # upper_bound
    i = min(max(j - 1, 0), N_NODES - 2)
    t = i + (r - R[i]) / (R[i + 1] - R[i])
    return math.exp(grid_log_e0() + t * grid_dlog())
