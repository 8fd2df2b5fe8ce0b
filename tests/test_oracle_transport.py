"""Pins for the oracle's transport: per-event energy ledger, Beer-Lambert
attenuation, CSDA slowing-down, RK4 against the exact helix (fourth-order
convergence and boundary snapping), a brute-force single step, and
invariance of whole-event results to thread count and event order."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads
from oracle import tables as T

PB = (82.0, 207.2, 11.35, 823.0)
LAR = (18.0, 39.948, 1.396, 188.0)


def ledger_residual(edep, led, prims, rows, n_rows):
    prim = np.zeros(n_rows)
    np.add.at(prim, rows, prims["T"])
    tot = edep.sum(1) + led["escaped"] + 2 * T.ME * (led["n_pair"].astype(float) - led["n_annih"].astype(float))
    return np.max(np.abs(tot - prim) / prim)


@pytest.mark.parametrize("wl", ["small", "field", "mixed"])
def test_energy_ledger_exact_per_event(wl):
    if wl == "small":
        w = workloads.small_electron_showers(300)
    elif wl == "field":
        w = workloads.electron_showers_1gev_field(8)
    else:
        w = workloads.mixed_cone_showers(12)
    pb = oracle.problem_for(w)
    tr, rows = oracle.tracks_from_primaries(w.primaries)
    edep, led, steps = pb.run_events(tr, rows, w.n_events, 4)
    assert steps == int(led["steps"].sum()) > 0
    assert ledger_residual(edep, led, w.primaries, rows, w.n_events) < 1e-9
    assert led["n_guard"].sum() == 0


def test_results_independent_of_threads_and_event_order():
    w = workloads.small_electron_showers(200)
    pb = oracle.problem_for(w)
    tr, rows = oracle.tracks_from_primaries(w.primaries)
    e1, l1, s1 = pb.run_events(tr, rows, w.n_events, 1)
    e4, l4, s4 = pb.run_events(tr, rows, w.n_events, 4)
    assert s1 == s4 and np.array_equal(e1, e4) and np.array_equal(l1, l4)
    perm = np.random.default_rng(0).permutation(len(tr))
    ep, lp, sp = pb.run_events(tr[perm], rows[perm], w.n_events, 3)
    assert sp == s1 and np.array_equal(ep, e1)


def test_beer_lambert_attenuation():
    # photons at a grid-node energy enter a 1 cm Pb slab along +z; the fraction
    # leaving through the back face on their first step is exp(-Sigma t), with
    # Sigma from the closed-form cross sections
    E = T.grid_energies()[80]           # 10 MeV node
    mat = T.Material(*PB)
    sig = mat.n_el * T.sigma_klein_nishina(E) + mat.n_at * T.sigma_photoelectric(E, mat.Z) + \
        T.sigma_pair_macro(E, mat.X0_cm)
    pb = oracle.Problem([0.0, 1.0], [0], 1e4, (0, 0, 0), [PB], 0.1, 7)
    n = 40000
    tr = np.zeros(n, dtype=oracle.TRACK_DTYPE)
    tr["event"] = 5
    tr["key"] = np.arange(n)
    tr["alive"] = 1
    tr["T"] = E
    tr["nl"] = -1.0
    tr["u"] = (0.0, 0.0, 1.0)
    res = pb.step(tr)
    through = np.sum((res["outcome"] == oracle.OUT_ESCAPE) & (res["face"] == oracle.F_ZHI))
    p = math.exp(-sig * 1.0)
    assert abs(through - n * p) <= 4 * math.sqrt(n * p * (1 - p))


@pytest.mark.parametrize("positron", [False, True])
def test_csda_slowing_down(positron):
    # no discrete processes: the lepton loses energy continuously until the
    # cut; all of its kinetic energy is deposited and its path length lies in
    # [R(T0) - R(Ec), R(T0)]
    Ec = 0.1
    pb = oracle.Problem([0.0, 100.0], [0], 1e4, (0, 0, 0), [PB], Ec, 3, no_discrete=True)
    T0 = 50.0
    t = np.zeros(1, dtype=oracle.TRACK_DTYPE)
    t["type"] = oracle.POSITRON if positron else oracle.ELECTRON
    t["alive"] = 1
    t["T"] = T0
    t["nl"] = -1.0
    t["r"] = (0.0, 0.0, 1.0)
    t["u"] = (0.0, 0.0, 1.0)
    R = pb.tables[0, T.T_RANGE_EP if positron else T.T_RANGE_EM]
    path = dep = 0.0
    n_annih = 0
    while t["alive"][0]:
        res = pb.step(t)
        path += res["step_len"][0]
        dep += res["edep"][0]
        n_annih += res["n_annih"][0]
        assert res["process"][0] == -1
    # Ec < m: the annihilation photons are emitted, not deposited
    assert dep == pytest.approx(T0, rel=1e-12)
    assert n_annih == (1 if positron else 0)
    assert path <= T.lookup(R, T0) * (1 + 1e-12)
    assert path >= T.lookup(R, T0) - T.lookup(R, Ec) - 1e-12


def _helix(r0, u0, kf, Bx, s):
    w = kf * Bx
    uy, uz = u0[1], u0[2]
    y = r0[1] + (uy * math.sin(w * s) - uz * math.cos(w * s) + uz) / w
    z = r0[2] + (uz * math.sin(w * s) + uy * math.cos(w * s) - uy) / w
    x = r0[0] + u0[0] * s
    u = (u0[0], uy * math.cos(w * s) + uz * math.sin(w * s), uz * math.cos(w * s) - uy * math.sin(w * s))
    return np.array([x, y, z]), np.array(u)


def test_rk4_fourth_order_against_exact_helix():
    B = np.array([1.0, 0.0, 0.0])
    u0 = np.array([0.3, 0.5, math.sqrt(1 - 0.34)])
    r0 = np.zeros(3)
    kf = -2.99792458 / 1.0     # electron with p = 1 MeV: radius ~ 0.33 cm
    L = 1.0
    errs = []
    for n in (16, 32, 64):
        h = L / n
        r, u = r0.copy(), u0.copy()
        for _ in range(n):
            r, u = oracle.rk4(r, u, h, kf, B)
        rex, _ = _helix(r0, u0, kf, 1.0, L)
        errs.append(np.linalg.norm(r - rex))
    assert 12 < errs[0] / errs[1] < 20 and 12 < errs[1] / errs[2] < 20


def test_field_boundary_snap_close_to_exact_helix_root():
    # an electron crossing a plane in a 1 T field: the snapped crossing point
    # lies within tolerance of the exact helix's crossing (found by bisection)
    pb = oracle.Problem([0.0, 0.3, 10.0], [0, 1], 20.0, (1.0, 0.0, 0.0), [PB, LAR], 0.1, 1, table_blob=np.zeros((2, 8, 181)))
    for uz in (0.9, 0.5, 0.2):
        u0 = np.array([0.1, math.sqrt(1 - 0.01 - uz * uz), uz])
        t = np.zeros(1, dtype=oracle.TRACK_DTYPE)
        t["type"] = oracle.ELECTRON
        t["T"] = 5.0
        t["r"] = (0.0, 0.0, 0.1)
        t["u"] = u0
        s, face, nsub = pb.propagate_field(t, 5.0)
        assert face == oracle.F_ZHI
        assert t["r"][0][2] == 0.3
        p = math.sqrt(5.0 * (5.0 + 2 * T.ME))
        kf = -2.99792458 / p
        lo, hi = 0.0, s * 1.5
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if _helix(np.array([0, 0, 0.1]), u0, kf, 1.0, mid)[0][2] < 0.3:
                lo = mid
            else:
                hi = mid
        rex, _ = _helix(np.array([0, 0, 0.1]), u0, kf, 1.0, lo)
        assert abs(s - lo) < 1e-4
        assert np.linalg.norm(t["r"][0] - rex) < 1e-4


def _bruteforce_exit(r, u, zlo, zhi, W):
    inside = lambda s: (zlo <= r[2] + s * u[2] <= zhi) and abs(r[0] + s * u[0]) <= W and abs(r[1] + s * u[1]) <= W  # noqa
    hi = 1.0
    while inside(hi):
        hi *= 2
    lo = 0.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if inside(mid):
            lo = mid
        else:
            hi = mid
    return lo


def test_single_step_brute_force():
    # one straight step, checked against an independent reconstruction:
    # exit distance by bisection on point-in-box, interaction length from the
    # uniform drawn through numpy's Philox, process from explicit cumulative
    # sums of the per-process cross sections
    w = workloads.small_electron_showers(1)
    pb = oracle.problem_for(w)
    z = pb.z_planes
    rng = np.random.default_rng(11)
    n = 400
    tr = np.zeros(n, dtype=oracle.TRACK_DTYPE)
    tr["event"] = rng.integers(0, 1000, n)
    tr["key"] = rng.integers(0, 2 ** 62, n)
    tr["type"] = rng.integers(0, 3, n)
    tr["slab"] = rng.integers(0, pb.n_slabs, n)
    tr["step"] = rng.integers(0, 50, n)
    tr["alive"] = 1
    tr["T"] = np.exp(rng.uniform(math.log(1.5), math.log(50.0), n))
    tr["nl"] = np.where(rng.uniform(size=n) < 0.5, -1.0, rng.exponential(1.0, n))
    ct = rng.uniform(-1, 1, n)
    ph = rng.uniform(0, 2 * math.pi, n)
    st = np.sqrt(1 - ct * ct)
    tr["u"] = np.stack([st * np.cos(ph), st * np.sin(ph), ct], 1)
    tr["r"][:, 0] = rng.uniform(-4.9, 4.9, n)
    tr["r"][:, 1] = rng.uniform(-4.9, 4.9, n)
    tr["r"][:, 2] = z[tr["slab"]] + rng.uniform(0.01, 0.99, n) * (z[tr["slab"] + 1] - z[tr["slab"]])
    before = tr.copy()
    res = pb.step(tr)
    procs = {0: [0, 1, 2], 1: [3, 5], 2: [4, 5]}
    n_inter = 0
    for i in range(n):
        b = before[i]
        mat = pb.slab_material[b["slab"]]
        j = 0
        nl = b["nl"]
        if nl < 0:
            w0 = oracle.philox4x64((b["key"], b["step"], 0, 0), (w.seed, b["event"]))
            nl = -math.log(workloads.unit(w0[0]))
            j = 1
        sig = sum(pb.xs(mat, p, b["T"]) for p in procs[int(b["type"])])
        s_int = nl / sig
        s_phys, loss = s_int, False
        if b["type"] != 0:
            R = T.lookup(pb.tables[mat, T.T_RANGE_EP if b["type"] == 2 else T.T_RANGE_EM], b["T"])
            s_loss = R if R <= 0.01 else max(0.01, 0.2 * R)
            if s_loss < s_int:
                s_phys, loss = s_loss, True
        s_geo = _bruteforce_exit(b["r"], b["u"], z[b["slab"]], z[b["slab"] + 1], 5.0)
        r = res[i]
        if s_geo <= s_phys * (1 - 1e-9):
            assert r["outcome"] in (oracle.OUT_BOUNDARY, oracle.OUT_ESCAPE, oracle.OUT_STOP), i
            assert r["step_len"] == pytest.approx(s_geo, rel=1e-9, abs=1e-12)
        elif s_geo >= s_phys * (1 + 1e-9):
            assert r["step_len"] == pytest.approx(s_phys, rel=1e-12)
            if loss:
                assert r["outcome"] in (oracle.OUT_LOSS, oracle.OUT_STOP)
            elif r["outcome"] != oracle.OUT_STOP:
                n_inter += 1
                Tpost = b["T"]
                w1 = oracle.philox4x64((b["key"], b["step"], j >> 2, 0), (w.seed, b["event"]))
                U1 = workloads.unit(w1[j & 3])
                if b["type"] != 0:
                    # post-loss energy is the pre-step energy minus the continuous deposit
                    Tpost = T.inverse_range(pb.tables[mat, T.T_RANGE_EP if b["type"] == 2 else T.T_RANGE_EM],
                                            T.lookup(pb.tables[mat, T.T_RANGE_EP if b["type"] == 2 else T.T_RANGE_EM],
                                                     b["T"]) - s_phys)
                xs = [pb.xs(mat, p, Tpost) for p in procs[int(b["type"])]]
                target = U1 * sum(xs)
                cum = np.cumsum(xs)
                expect = procs[int(b["type"])][int(np.argmax(target < cum))]
                assert r["process"] == expect, i
    assert n_inter > 20


# ---------------------------------------------------------------- flip diagnosis hooks
def test_margin_recording_changes_nothing_and_trace_equals_run():
    """Recording decision margins reads values only: single steps and whole
    event histories are bit-identical with and without it, and the trace of
    an event sums to orc_run_events' deposits, ledger and step count."""
    import numpy as np
    from tests.gpu_helpers import random_states
    w = workloads.electron_showers_1gev_field(2)
    pb = oracle.problem_for(w)
    st = random_states(w, 2000, np.random.default_rng(3))
    a, b = st.copy(), st.copy()
    ra = pb.step(a)
    rb, m = pb.step_margins(b)
    assert np.array_equal(a, b) and np.array_equal(ra, rb)
    assert np.all(m["margin"] >= 0) and np.all(m["n_notes"] > 0)
    tr, rows = oracle.tracks_from_primaries(w.primaries[:1])
    t = pb.trace_event(tr)
    e, led, steps = pb.run_events(tr, rows[:1] * 0, 1, 1)
    assert len(t) == steps == led["steps"][0]
    dep = np.zeros(pb.n_slabs)
    np.add.at(dep, t["res"]["dep_slab"], t["res"]["edep"])
    assert np.array_equal(dep, e[0])
    assert t["res"]["escaped"].sum() == led["escaped"][0]
    assert t["res"]["n_pair"].sum() == led["n_pair"][0]
    # history order: every step's track was created by an earlier step
    seen = {int(tr["key"][0])}
    for r in t:
        assert int(r["pre"]["key"]) in seen
        for k in range(int(r["res"]["n_sec"])):
            seen.add(int(r["res"]["sec"][k]["key"]))


def test_margin_of_a_step_at_a_threshold():
    """A positron 1e-9 above the cut: the smallest margin of its step is the
    cut / process-threshold decision, at 1e-9 relative; a step far from every
    threshold has a much larger margin."""
    import numpy as np
    w = workloads.small_electron_showers(1)
    pb = oracle.problem_for(w)
    t = np.zeros(2, dtype=oracle.TRACK_DTYPE)
    t["type"] = oracle.POSITRON
    t["T"] = [w.ecut * (1 + 1e-9), 5.0]
    t["nl"] = [-1.0, 0.3]
    t["r"] = [(0.1, 0.2, 0.05), (0.1, 0.2, 0.05)]
    t["u"] = [(0.0, 0.6, 0.8), (0.0, 0.6, 0.8)]
    t["alive"] = 1
    _, m = pb.step_margins(t)
    assert m["margin"][0] == pytest.approx(1e-9, rel=1e-3)
    assert oracle.MARGIN_KINDS[m["kind"][0]] in ("cut at step start", "process threshold")
    assert m["margin"][1] > 1e-6
