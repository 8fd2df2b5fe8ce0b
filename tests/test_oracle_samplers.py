"""Pins for the oracle's final-state samplers: chi-square of each sampled
spectrum against its differential cross section (integrated independently by
quadrature), and exact energy-momentum conservation of the two-body
kinematics."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
from oracle import tables as T

N = 20000
NB = 25


def _problem(ecut):
    st_z = np.array([0.0, 1000.0])
    zeros = np.zeros((2, 8, 181))
    return oracle.Problem(st_z, [0], 500.0, (0, 0, 0), [(82.0, 207.2, 11.35, 823.0), (18.0, 39.948, 1.396, 188.0)],
                          ecut, 1, table_blob=zeros)


def _tracks(typ, Tk, n, event=3):
    t = np.zeros(n, dtype=oracle.TRACK_DTYPE)
    t["event"] = event
    t["key"] = np.arange(n, dtype=np.uint64) * np.uint64(2654435761) + np.uint64(17)
    t["type"] = typ
    t["slab"] = 0
    t["alive"] = 1
    t["T"] = Tk
    t["nl"] = -1.0
    t["r"] = (0.0, 0.0, 1.0)
    th = np.linspace(0.1, 2.9, n)
    t["u"] = np.stack([np.sin(th) * np.cos(3 * th), np.sin(th) * np.sin(3 * th), np.cos(th)], axis=1)
    return t


def _chi2(samples, lo, hi, pdf, log_bins=False):
    edges = np.geomspace(lo, hi, NB + 1) if log_bins else np.linspace(lo, hi, NB + 1)
    probs = np.array([integrate.quad(pdf, a, b, epsrel=1e-12)[0] for a, b in zip(edges[:-1], edges[1:])])
    probs /= probs.sum()
    counts, _ = np.histogram(samples, bins=edges)
    assert counts.sum() == len(samples)
    return stats.chisquare(counts, probs * counts.sum()).pvalue


@pytest.mark.parametrize("E", [0.05, 0.511, 5.11, 511.0])
def test_compton_energy_spectrum_chi2(E):
    pb = _problem(1e-9)
    tr = _tracks(oracle.GAMMA, E, N)
    u0 = tr["u"].copy()
    res = pb.interact(tr, oracle.P_COMPTON)
    eps = tr["T"] / E
    k = E / T.ME
    e0 = 1 / (1 + 2 * k)
    p = _chi2(eps, e0, 1.0, lambda x: T.dsigma_klein_nishina_deps(E, x), log_bins=True)
    assert p > 1e-3
    # photon scattering angle follows the Compton formula
    cos_expect = 1 - (1 - eps) / (k * eps)
    assert np.allclose(np.sum(u0 * tr["u"], axis=1), cos_expect, atol=1e-12)
    # momentum conservation with the electron
    for i in range(0, N, 97):
        if res["n_sec"][i] == 0:
            continue
        s = res["sec"][i][0]
        pe = math.sqrt(s["T"] * (s["T"] + 2 * T.ME))
        miss = E * u0[i] - tr["T"][i] * tr["u"][i] - pe * s["u"]
        assert np.linalg.norm(miss) <= 1e-12 * E
        assert s["T"] + tr["T"][i] == pytest.approx(E, rel=1e-15)


@pytest.mark.parametrize("E", [2.0, 10.0, 1000.0])
def test_pair_energy_sharing_chi2(E):
    pb = _problem(1e-9)
    tr = _tracks(oracle.GAMMA, E, N)
    res = pb.interact(tr, oracle.P_PAIR)
    assert np.all(res["n_sec"] == 2) and np.all(res["n_pair"] == 1)
    pos = res["sec"][:, 1]
    assert np.all(pos["type"] == oracle.POSITRON)
    x = (pos["T"] + T.ME) / E
    a = T.ME / E
    p = _chi2(x, a, 1 - a, lambda v: 1 - 4 / 3 * v * (1 - v))
    assert p > 1e-3
    ele = res["sec"][:, 0]
    assert np.allclose(ele["T"] + pos["T"] + 2 * T.ME, E, rtol=1e-14)


@pytest.mark.parametrize("Tk,Ec", [(10.0, 0.1), (1000.0, 0.1)])
def test_brems_photon_spectrum_chi2(Tk, Ec):
    pb = _problem(Ec)
    tr = _tracks(oracle.ELECTRON, Tk, N)
    res = pb.interact(tr, oracle.P_BREMS)
    g = res["sec"][:, 0]
    assert np.all(g["type"] == oracle.GAMMA)
    E = Tk + T.ME
    y = g["T"] / E
    p = _chi2(y, Ec / E, Tk / E, lambda v: (4 / 3 - 4 / 3 * v + v * v) / v, log_bins=True)
    assert p > 1e-3


@pytest.mark.parametrize("proc,typ,hi", [(oracle.P_MOLLER, oracle.ELECTRON, 0.5), (oracle.P_BHABHA, oracle.POSITRON, 1.0)])
@pytest.mark.parametrize("Tk", [1.0, 100.0])
def test_delta_ray_spectrum_chi2_and_kinematics(proc, typ, hi, Tk):
    Ec = 0.1
    pb = _problem(Ec)
    tr = _tracks(typ, Tk, N)
    u0 = tr["u"].copy()
    res = pb.interact(tr, proc)
    d = res["sec"][:, 0]
    ok = d["type"] == oracle.ELECTRON
    assert ok.mean() > 0.999
    eps = d["T"][ok] / Tk
    pdf = (lambda e: T.dsigma_moller_deps(Tk, e)) if proc == oracle.P_MOLLER else (lambda e: T.dsigma_bhabha_deps(Tk, e))
    assert _chi2(eps, Ec / Tk, hi, pdf, log_bins=True) > 1e-3
    # momentum conservation for survivors: p u = p_d u_d + p_n u_n
    p = math.sqrt(Tk * (Tk + 2 * T.ME))
    for i in np.nonzero(ok & (tr["alive"] == 1))[0][::53]:
        pd = math.sqrt(d["T"][i] * (d["T"][i] + 2 * T.ME))
        Tn = tr["T"][i]
        pn = math.sqrt(Tn * (Tn + 2 * T.ME))
        miss = p * u0[i] - pd * d["u"][i] - pn * tr["u"][i]
        assert np.linalg.norm(miss) <= 1e-12 * p
        assert Tn + d["T"][i] == pytest.approx(Tk, rel=1e-15)


def test_annihilation_at_rest_isotropic_back_to_back():
    pb = _problem(0.1)
    tr = _tracks(oracle.POSITRON, 0.05, N)   # below the cut: stops at its first step
    res = pb.step(tr)
    assert np.all(res["outcome"] == oracle.OUT_STOP) and np.all(res["n_annih"] == 1)
    assert np.all(res["n_sec"] == 2)
    g1, g2 = res["sec"][:, 0], res["sec"][:, 1]
    assert np.allclose(g1["T"], T.ME) and np.allclose(g2["T"], T.ME)
    assert np.allclose(g1["u"], -g2["u"], atol=0)
    assert np.allclose(res["edep"], 0.05)
    assert stats.kstest(g1["u"][:, 2], "uniform", args=(-1, 2)).pvalue > 1e-3
    phi = np.arctan2(g1["u"][:, 1], g1["u"][:, 0])
    assert stats.kstest(phi, "uniform", args=(-math.pi, 2 * math.pi)).pvalue > 1e-3
    # the two photons carry distinct keys
    assert len(set(g1["key"].tolist()) | set(g2["key"].tolist())) == 2 * N


def test_annihilation_deposited_when_rest_mass_below_cut():
    pb = _problem(1.0)
    tr = _tracks(oracle.POSITRON, 0.5, 10)
    res = pb.step(tr)
    assert np.all(res["n_sec"] == 0)
    assert np.allclose(res["edep"], 0.5 + 2 * T.ME, rtol=1e-15)
