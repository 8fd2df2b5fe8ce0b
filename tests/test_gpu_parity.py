"""GPU parity of the HIP step loop against the CPU oracle.

* device-built physics tables equal the oracle's tables;
* the device stable sort equals numpy's stable argsort (bit-exact);
* one step of injected states equals the oracle's single step (FP64 1e-12;
  mixed FP32 1e-5 relative to the pre-step energy);
* whole showers: per-event integer counts equal, per-event deposits paired to
  1e-9, per-layer means within 3 sigma, exact energy ledger;
* results do not depend on sort policy, charged/neutral partitioning, the
  field-substep cap (pause and resume) or the slot count.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_helpers import (assert_events_match, event_energy, layer_sums, ledger_int_mismatch, random_states,
                               session_for, to_lib_tracks)

pytestmark = pytest.mark.gpu


_ledger_equal_int = ledger_int_mismatch


# ----------------------------------------------------------------------------- tables
@pytest.mark.parametrize("ecut", [0.1, 1.0])
def test_device_tables_match_oracle(ecut):
    w = workloads.small_electron_showers(1)
    w.ecut = ecut
    s = session_for(w, n_slots=1024)
    dev = s.read_tables()
    ref = oracle.tables.build_tables([oracle.tables.Material(*m) for m in w.stack.materials], ecut)
    assert dev.shape == ref.shape
    zero = ref == 0.0
    assert np.array_equal(dev == 0.0, zero)
    # 1e-12 relative, with an absolute floor of 1e-10 of each table's largest
    # value: entries a rounding away from a threshold (node energy at the cut)
    # and the Klein-Nishina closed form at a few keV (cancellation) are only
    # defined to that level on either side
    scale = np.abs(ref).max(axis=2, keepdims=True)
    err = np.abs(dev - ref)
    ok = err <= 1e-12 * np.abs(ref) + 1e-10 * scale
    bad = np.argwhere(~ok)
    report = [(tuple(b), dev[tuple(b)], ref[tuple(b)]) for b in bad[:8]]
    s.close()
    assert ok.all(), report
    # away from thresholds and above 0.1 MeV the tables agree to 1e-12 relative
    E = oracle.tables.grid_energies()
    sel = (E >= 0.1) & (E >= 1.2 * 2 * ecut)
    for t in range(8):
        r, d_ = ref[:, t, sel], dev[:, t, sel]
        nz = r != 0
        assert (np.abs(d_[nz] - r[nz]) / np.abs(r[nz])).max() < 1e-12, t


# ----------------------------------------------------------------------------- sort
@pytest.mark.parametrize("n", [1, 63, 4096, 4097, 100_003, 1 << 20, (1 << 20) + 1])
@pytest.mark.parametrize("policy,nb", [("partition", 16), ("radix", 128)])
def test_sort_permutation_bit_exact(n, policy, nb):
    w = workloads.small_electron_showers(1)
    s = session_for(w, n_slots=1024)
    rng = np.random.default_rng(n + nb)
    for dist in ("uniform", "skewed", "constant"):
        if dist == "uniform":
            keys = rng.integers(0, nb, n)
        elif dist == "skewed":
            keys = np.minimum(rng.geometric(0.4, n) - 1, nb - 1)
        else:
            keys = np.full(n, nb - 1)
        perm = s.sort(keys.astype(np.uint8), policy)
        assert np.array_equal(perm, np.argsort(keys, kind="stable").astype(np.uint32)), dist
    s.close()


# ----------------------------------------------------------------------------- one step
def _step_compare(w, n, precision, seed, tol, types=(0, 1, 2), e_max=1000.0, msc=False, steps=(0, 200),
                  return_margins=False):
    rng = np.random.default_rng(seed)
    f32 = precision == "mixed"
    states = random_states(w, n, rng, types=types, e_max=e_max, f32=f32, steps=steps)
    s = session_for(w, n_slots=n, precision=precision, max_events=n, max_substeps=0,
                    n_initializers=4 * n, msc=msc)
    rows = np.array([s.register_event(int(e)) for e in states["event"]], dtype=np.uint32)
    s.inject(to_lib_tracks(states, rows))
    s.iterate(1, no_init=True)
    got = s.read_tracks(n)
    sec = s.read_secondaries()
    edep, led, ev = s.read_all()
    s.close()

    pb = oracle.problem_for(w, msc=msc)
    ref_t = states.copy()
    res, margins = pb.step_margins(ref_t)

    bad = []
    worst = 0.0
    sec_by_row = {}
    for k in range(len(sec)):
        sec_by_row.setdefault(int(sec["row"][k]), []).append(sec[k])
    for i in range(n):
        r, g, o = rows[i], got[i], ref_t[i]
        T0 = states["T"][i]
        alive_ref = bool(o["alive"])
        alive_gpu = g["type"] >= 0
        errs = []
        if alive_ref != alive_gpu:
            bad.append((i, "alive", alive_ref, alive_gpu, res[i]["outcome"]))
            continue
        if alive_ref:
            if g["slab"] != o["slab"] or g["step"] != o["step"] or g["type"] != o["type"]:
                bad.append((i, "int", (g["slab"], g["step"]), (o["slab"], o["step"])))
                continue
            errs.append(("T", abs(g["T"] - o["T"]) / T0))
            errs.append(("u", np.abs(g["u"] - o["u"]).max()))
            errs.append(("r", np.abs(g["r"] - o["r"]).max() / max(np.linalg.norm(o["r"]), 1.0)))
            if (o["nl"] < 0) != (g["nl"] < 0):
                bad.append((i, "nl-unset", g["nl"], o["nl"]))
                continue
            if o["nl"] >= 0:
                errs.append(("n_lambda", abs(g["nl"] - o["nl"]) / max(abs(o["nl"]), 1.0)))
        # tallies of this track's row
        e_gpu = edep[r]
        e_ref = np.zeros_like(e_gpu)
        e_ref[res[i]["dep_slab"]] = res[i]["edep"]
        errs.append(("deposit", np.abs(e_gpu - e_ref).max() / T0))
        errs.append(("escaped", abs(led[r]["escaped"] - res[i]["escaped"]) / T0))
        if led[r]["n_pair"] != res[i]["n_pair"] or led[r]["n_annih"] != res[i]["n_annih"]:
            bad.append((i, "pair/annih"))
            continue
        if alive_ref is False and led[r]["steps"] != o["step"]:
            bad.append((i, "steps", led[r]["steps"], o["step"]))
            continue
        # secondaries matched by key
        gs = sorted(sec_by_row.get(int(r), []), key=lambda x: int(x["key"]))
        os_ = sorted(list(res[i]["sec"][: res[i]["n_sec"]]), key=lambda x: int(x["key"]))
        if len(gs) != len(os_):
            bad.append((i, "n_sec", len(gs), len(os_), res[i]["process"]))
            continue
        for a, b in zip(gs, os_):
            if a["key"] != b["key"] or a["type"] != b["type"] or a["slab"] != b["slab"]:
                bad.append((i, "sec-int"))
                break
            errs.append(("secondary T", abs(a["T"] - b["T"]) / T0))
            errs.append(("secondary u", np.abs(a["u"] - b["u"]).max()))
            errs.append(("secondary r", np.abs(a["r"] - b["r"]).max() / max(np.linalg.norm(b["r"]), 1.0)))
        what, e = max(errs, key=lambda x: x[1]) if errs else ("", 0.0)
        worst = max(worst, e)
        if e > tol:
            bad.append((i, "tol", e, what, res[i]["outcome"], res[i]["process"]))
    if return_margins:
        return bad, worst, margins, states
    return bad, worst


@pytest.mark.parametrize("wl", ["nofield", "field"])
def test_single_step_parity_at_the_step_guard(wl):
    """Tracks whose step ends past the step limit (10^6): the guard stops them
    after the along-step or after the interaction; a positron stopped by the
    guard annihilates at rest with the counted step's index, adding no step."""
    w = workloads.small_electron_showers(1) if wl == "nofield" else workloads.electron_showers_1gev_field(1)
    bad, worst = _step_compare(w, 20000, "f64", seed=11, tol=1e-12, e_max=50.0, steps=(999_999, 1_000_001))
    print("worst", worst, "mismatches", len(bad), bad[:5])
    assert not bad, bad[:10]


@pytest.mark.parametrize("wl", ["nofield", "field"])
def test_single_step_parity_fp64(wl):
    w = workloads.small_electron_showers(1) if wl == "nofield" else workloads.electron_showers_1gev_field(1)
    bad, worst = _step_compare(w, 30000, "f64", seed=7 if wl == "nofield" else 8, tol=1e-12)
    print("worst", worst, "mismatches", len(bad), bad[:5])
    assert not bad, bad[:10]


@pytest.mark.parametrize("wl", ["nofield", "field"])
def test_single_step_parity_mixed(wl):
    w = workloads.small_electron_showers(1) if wl == "nofield" else workloads.electron_showers_1gev_field(1)
    n = 30000
    bad, worst, margins, states = _step_compare(w, n, "mixed", seed=17, tol=1e-5, return_margins=True)
    _assert_fp32_flips(w, bad, worst, margins, states, n)


def _draw_resolution(w, st):
    """Relative difference of the interaction length drawn by a step in FP32
    and in FP64 from the same Philox word: the FP32 uniform keeps the word's
    top 23 bits, so -ln U differs by up to 2^-24 / U, which is large for
    small U.  Zero when the step draws no interaction length."""
    if st["nl"] >= 0:
        return 0.0
    wd = int(oracle.philox4x64([int(st["key"]), int(st["step"]), 0, 0], [w.seed, int(st["event"])])[0])
    u64 = ((wd >> 12) + 0.5) * 2.0 ** -52
    u32 = float(np.float32(((wd >> 41) + 0.5) * 2.0 ** -23))
    n64, n32 = -np.log(u64), -np.log(u32)
    return abs(n32 - n64) / max(n64, 1.0)


def _assert_fp32_flips(w, bad, worst, margins, states, n):
    """Mixed precision against the FP64 oracle.  A step outside 1e-5 (of any
    kind: a state, tally or secondary outside tolerance, a different
    process, end of step or secondary) is sorted by cause:
    * a flip: the oracle took one of the step's discrete decisions within
      1e-5 of its threshold, which FP32 arithmetic can take the other way;
      at most 5e-4 of the steps (at least 3);
    * draw resolution: the step drew its interaction length from a uniform
      small enough that the FP32 uniform's 23 bits change -ln U by more than
      1e-6 (the FP32 reading of the random numbers: same word, fewer bits),
      which moves the step's end without any decision near its threshold;
      about 1e-3 of the draws, at most 2e-3 of the steps;
    * conditioning: a state, tally or secondary value (no structural
      difference) off by less than 1e-3, where the step amplifies FP32
      rounding: a direction stored in FP32 enters the rotation of the next
      sampled angle, whose azimuth frame turns fast near the z axis (the
      rotation divides by sqrt(1 - u_z^2)); the energy after a step close to
      the end of the range is the difference of nearly equal ranges; a
      process selection at a margin of 1e-4 follows from such an energy;
      at most 5e-4 of the steps (at least 3).
    Anything else (a structural difference away from any threshold, or an
    error of 1e-3 or more) fails.  Measured on 30 000 (20 000 with multiple
    scattering) steps: no field 9 (all draw resolution); field 11 (3 flips,
    6 draw resolution, 2 directions at 1.5e-5); with multiple scattering 7
    (6 draw resolution, 1 direction) and, in the field, 15 (6 flips, 2 draw
    resolution, 7 conditioning, the largest 2.4e-4)."""
    flips, resolution, conditioning, unexplained = [], [], [], []
    for b in bad:
        i = b[0]
        mg, kind = float(margins[i]["margin"]), oracle.MARGIN_KINDS[int(margins[i]["kind"])]
        dr = _draw_resolution(w, states[i])
        rec = (i, b[1:4], mg, kind, dr)
        if mg < 1e-5:
            flips.append(rec)
        elif dr > 1e-6:
            resolution.append(rec)
        elif b[1] == "tol" and b[2] < 1e-3:
            conditioning.append(rec)
        else:
            unexplained.append(rec)
    print("worst", worst, "mismatches", len(bad), "flips", len(flips), "draw resolution", len(resolution),
          "conditioning", len(conditioning), "unexplained", len(unexplained),
          (unexplained or flips or conditioning or resolution)[:6])
    assert not unexplained, unexplained[:10]
    assert len(flips) <= max(3, int(5e-4 * n)), flips[:10]
    assert len(resolution) <= max(3, int(2e-3 * n)), resolution[:10]
    assert len(conditioning) <= max(3, int(5e-4 * n)), conditioning[:10]


# ----------------------------------------------------------------------------- showers
def _run_lib(w, **kw):
    s = session_for(w, **kw)
    s.push(w.primaries)
    c = s.run(max_iterations=200000)
    edep, led = s.tallies_by_event(np.arange(w.n_events))
    s.close()
    return edep, led, c


def _run_oracle(w, threads=8):
    pb = oracle.problem_for(w)
    tr, rows = oracle.tracks_from_primaries(w.primaries)
    return pb.run_events(tr, rows, w.n_events, threads)


def test_small_showers_end_to_end_parity():
    w = workloads.small_electron_showers(1000)
    edep, led, c = _run_lib(w)
    e_ref, l_ref, steps = _run_oracle(w)
    assert c["overflow"] == 0
    assert c["steps"] == steps
    assert _ledger_equal_int(led, l_ref) is None
    rel = np.abs(edep - e_ref).max(1) / w.primaries["T"]
    assert rel.max() < 1e-9, rel.max()
    assert np.allclose(led["escaped"], l_ref["escaped"], rtol=1e-9, atol=1e-9)
    # per-layer means within 3 sigma
    lg, lr = layer_sums(edep), layer_sums(e_ref)
    sig = np.sqrt(lg.var(0) / len(lg) + lr.var(0) / len(lr))
    assert np.all(np.abs(lg.mean(0) - lr.mean(0)) <= 3 * sig + 1e-12)
    # exact energy ledger
    tot = edep.sum(1) + led["escaped"] + 2 * 0.51099895 * (led["n_pair"].astype(float) - led["n_annih"])
    assert np.max(np.abs(tot - w.primaries["T"]) / w.primaries["T"]) < 1e-9


def test_field_showers_parity_and_policy_invariance():
    w = workloads.electron_showers_1gev_field(40, n_slots=1 << 15)
    e_ref, l_ref, steps = _run_oracle(w)
    base = None
    for policy, part, sub, slots in [("none", False, 10, 1 << 15), ("partition", True, 10, 1 << 15),
                                     ("radix", False, 1, 1 << 13), ("none", True, 0, 1 << 16),
                                     ("partition", False, 3, 5000), ("queue", False, 10, 1 << 15),
                                     ("queue", True, 2, 3000), ("radix", True, 10, 1 << 14)]:
        edep, led, c = _run_lib(w, n_slots=slots, sort_policy=policy, init_partition=part, max_substeps=sub)
        tag = (policy, part, sub, slots)
        assert c["overflow"] == 0, tag
        assert c["steps"] == steps, (tag, c["steps"], steps)
        assert _ledger_equal_int(led, l_ref) is None, (tag, _ledger_equal_int(led, l_ref))
        rel = np.abs(edep - e_ref).max(1) / w.primaries["T"]
        assert rel.max() < 1e-9, (tag, rel.max())
        if base is None:
            base = edep
        assert np.abs(edep - base).max() < 1e-9 * 1000.0, tag


def test_mixed_precision_per_layer_error():
    w = workloads.mixed_cone_showers(200, n_slots=1 << 16)
    edep, led, c = _run_lib(w, precision="mixed")
    e_ref, l_ref, steps = _run_oracle(w)
    lg, lr = layer_sums(edep).mean(0), layer_sums(e_ref).mean(0)
    big = lr >= 0.01 * lr.sum()
    err = np.abs(lg[big] - lr[big]) / lr[big]
    print("mixed per-layer max rel err", err.max(), "steps", c["steps"], steps)
    assert err.max() <= 0.005


def test_tuning_does_not_change_results():
    w = workloads.electron_showers_1gev_field(20, n_slots=1 << 14)
    e_ref, l_ref, steps = _run_oracle(w)
    s = session_for(w, sort_policy="partition", graph_iterations=4)
    for tuning in [dict(sort_policy="radix", tail_threshold=3000, block={"pre_step": 64, "along_field": 512}),
                   dict(sort_policy="queue", tail_threshold=0, block={"along_neutral": 128, "compton": 448}),
                   dict(sort_policy="none", tail_threshold=100000, block={"bremsstrahlung": 64}),
                   dict(sort_policy="partition", tail_threshold=0, reuse_parent_slot=True),
                   dict(sort_policy="queue", reuse_parent_slot=True, drain_threshold=3000, drain_steps=50),
                   dict(sort_policy="partition", reuse_parent_slot=False, fuse_interactions=True),
                   dict(sort_policy="queue", tail_threshold=0, block={"along_field": 64}),
                   dict(sort_policy="queue", fuse_interactions=True, drain_threshold=0),
                   dict(sort_policy="none", fuse_interactions=True, block={"interactions": 128}),
                   dict(sort_policy="radix", tail_threshold=2000, fuse_interactions=True, reuse_parent_slot=True),
                   dict(sort_policy="partition", fuse_along=False, fuse_interactions=True),
                   dict(sort_policy="none", fuse_along=False, block={"along_field": 128}),
                   dict(sort_policy="partition", fuse_along=True, block={"along_field": 512}, tail_threshold=0),
                   dict(sort_policy="partition", phase_sort=(0, 0xFFFFFFFF)),
                   dict(sort_policy="radix", phase_sort=(0xFFFFFFFF, 0)),
                   dict(sort_policy="partition", phase_sort=(0x0007FFFF, 0xFFFFFFFF))]:
        s.set_tuning(**tuning)
        s.push(w.primaries)
        c = s.run()
        edep, led = s.tallies_by_event(np.arange(w.n_events))
        for e in range(w.n_events):
            s.release(e)
        assert _ledger_equal_int(led, l_ref) is None, tuning
        assert np.abs(edep - e_ref).max() <= 1e-9 * 1000.0, tuning
    s.close()


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_fused_along_steps_match_separate_launches_and_oracle(precision):
    """Photon and field along-steps in one launch (tuning fuse_along, one
    stream): the same per-track code as the two separate kernels, so the
    results equal theirs (integer ledgers exactly, deposits to 1e-12 of the
    event energy) and, in FP64, the oracle's, for every sort policy; masked
    (policy none) each slot takes the along-step of its type.  Few slots
    (2^12) keep both ranges longer than the grid, so threads take several
    field rounds and photon chunks."""
    w = workloads.electron_showers_1gev_field(40, n_slots=1 << 12)
    e0 = event_energy(w)
    if precision == "f64":
        e_ref, l_ref, steps = _run_oracle(w)
    for policy in ("partition", "none", "radix"):
        res = {}
        for fused in (True, False):
            s = session_for(w, precision=precision, sort_policy=policy, init_partition=True, graph_iterations=4,
                            streams=1)
            s.set_tuning(fuse_interactions=True, fuse_along=fused)
            s.push(w.primaries)
            c = s.run(max_iterations=1_000_000)
            res[fused] = (c, *s.tallies_by_event(np.arange(w.n_events)))
            s.close()
        (c1, e1, l1), (c0, ea, la) = res[True], res[False]
        assert c1["steps"] == c0["steps"] and c1["overflow"] == 0, policy
        assert _ledger_equal_int(l1, la) is None, policy
        assert np.all(np.abs(e1 - ea).max(1) <= 1e-12 * e0), policy
        assert c1["work"]["along_neutral"] == c0["work"]["along_neutral"] > 0, policy
        if precision == "f64":
            assert c1["steps"] == steps
            assert _ledger_equal_int(l1, l_ref) is None, policy
            assert np.all(np.abs(e1 - e_ref).max(1) <= 1e-9 * e0), policy


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_drain_mode_matches_step_loop_and_oracle(precision):
    """The block-local drain of the last tracks gives the step loop's
    results: every track is stepped by the same per-track code with the same
    keyed random numbers, whatever the threshold, the per-launch round budget
    (small budgets stop blocks mid-shower and hand their stacks back) or the
    slot count.  Draining from the first iteration (threshold 0xFFFFFFFF)
    puts whole 1 GeV showers into one block, so its stack overflows into the
    initializer buffer; the other thresholds start the drain in the tail."""
    w = workloads.electron_showers_1gev_field(30, n_slots=1 << 15)
    ref_e, ref_l, ref_c = _run_lib(w, precision=precision, sort_policy="partition", graph_iterations=4)
    if precision == "f64":
        e_or, l_or, steps = _run_oracle(w)
        assert ref_c["steps"] == steps
        assert _ledger_equal_int(ref_l, l_or) is None
    for thr, budget, slots in [(0xFFFFFFFF, 4096, 1 << 15), (4000, 3, 1 << 15), (20000, 64, 5000), (1000, 100000, 1 << 16)]:
        s = session_for(w, n_slots=slots, precision=precision, sort_policy="partition", graph_iterations=4)
        s.set_tuning(drain_threshold=thr, drain_steps=budget)
        s.push(w.primaries)
        c = s.run(max_iterations=1_000_000)
        edep, led = s.tallies_by_event(np.arange(w.n_events))
        s.close()
        tag = (precision, thr, budget, slots)
        assert c["overflow"] == 0, tag
        assert c["work"]["drain"] > 0, tag
        assert c["steps"] == ref_c["steps"], (tag, c["steps"], ref_c["steps"])
        assert _ledger_equal_int(led, ref_l) is None, (tag, _ledger_equal_int(led, ref_l))
        scale = np.abs(ref_e).max(1, keepdims=True)
        assert np.all(np.abs(edep - ref_e) <= 1e-12 * scale + 1e-300), tag


@pytest.mark.parametrize("precision,wl", [("f64", "nofield"), ("f64", "field"), ("mixed", "nofield"),
                                          ("mixed", "field")])
def test_single_step_parity_with_multiple_scattering(precision, wl):
    w = workloads.small_electron_showers(1) if wl == "nofield" else workloads.electron_showers_1gev_field(1)
    n = 20000
    tol = 1e-12 if precision == "f64" else 1e-5
    bad, worst, margins, states = _step_compare(w, n, precision, seed=23, tol=tol, types=(1, 2), msc=True,
                                                return_margins=True)
    if precision == "f64":
        print("worst", worst, "mismatches", len(bad), bad[:5])
        assert not bad, bad[:10]
    else:
        _assert_fp32_flips(w, bad, worst, margins, states, n)


def test_showers_with_multiple_scattering_match_oracle():
    w = workloads.electron_showers_1gev_field(30, n_slots=1 << 15)
    pb = oracle.problem_for(w, msc=True)
    tr, rows = oracle.tracks_from_primaries(w.primaries)
    e_ref, l_ref, steps = pb.run_events(tr, rows, w.n_events, 8)
    e_off, _, steps_off = _run_oracle(w)
    assert steps != steps_off
    for policy, drain in (("partition", 0), ("none", 0), ("partition", 65536)):
        s = session_for(w, sort_policy=policy, graph_iterations=4, msc=True)
        if drain:
            s.set_tuning(drain_threshold=drain)
        s.push(w.primaries)
        c = s.run()
        edep, led = s.tallies_by_event(np.arange(w.n_events))
        s.close()
        assert c["steps"] == steps, (policy, drain, c["steps"], steps)
        assert_events_match(w, edep, led, e_ref, l_ref, (policy, drain), msc=True)
