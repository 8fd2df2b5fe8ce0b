"""Shared helpers for the GPU parity tests: build a library session and the
oracle problem for the same workload, and convert track records."""
import math

import numpy as np

import oracle
import workloads
from tests import flip_diagnosis as fd


def session_for(workload, n_slots=None, precision="f64", max_events=None, **kw):
    from paper_2503_17608_amd import emstep
    st = workload.stack
    s = emstep.Session(n_slots or workload.n_slots, precision=precision,
                       max_events=max_events or max(workload.n_events, 1), max_slabs=st.n_slabs,
                       max_materials=len(st.materials), seed=workload.seed, **kw)
    s.load(st.z_planes, st.slab_material, st.half_width, st.B, st.materials, workload.ecut)
    return s


def random_states(workload, n, rng, types=(0, 1, 2), e_max=1000.0, f32=False, steps=(0, 200)):
    """Random single-track states inside the stack (some on planes / near walls);
    step counts uniform in [steps[0], steps[1])."""
    st = workload.stack
    z = st.z_planes
    W = st.half_width
    t = np.zeros(n, dtype=oracle.TRACK_DTYPE)
    t["event"] = rng.integers(0, 2 ** 40, n)
    t["key"] = rng.integers(0, 2 ** 63, n)
    t["type"] = rng.choice(types, n)
    t["slab"] = rng.integers(0, st.n_slabs, n)
    t["step"] = rng.integers(steps[0], steps[1], n)
    t["alive"] = 1
    t["T"] = np.exp(rng.uniform(math.log(workload.ecut * 1.0001), math.log(e_max), n))
    t["nl"] = np.where(rng.uniform(size=n) < 0.5, -1.0, rng.exponential(1.0, n))
    ct = rng.uniform(-1, 1, n)
    ph = rng.uniform(0, 2 * math.pi, n)
    sn = np.sqrt(1 - ct * ct)
    t["u"] = np.stack([sn * np.cos(ph), sn * np.sin(ph), ct], 1)
    sl = t["slab"]
    frac = rng.uniform(0.0, 1.0, n)
    on_lo = rng.uniform(size=n) < 0.1
    frac[on_lo] = 0.0
    t["r"][:, 2] = z[sl] + frac * (z[sl + 1] - z[sl])
    t["r"][on_lo, 2] = z[sl[on_lo]]
    t["r"][:, 0] = rng.uniform(-0.98 * W, 0.98 * W, n)
    t["r"][:, 1] = rng.uniform(-0.98 * W, 0.98 * W, n)
    if f32:
        t["T"] = t["T"].astype(np.float32).astype(np.float64)
        t["nl"] = t["nl"].astype(np.float32).astype(np.float64)
        t["u"] = t["u"].astype(np.float32).astype(np.float64)
        t["T"] = np.maximum(t["T"], np.nextafter(np.float32(workload.ecut), np.float32(1e9)).astype(np.float64))
    return t


def to_lib_tracks(orc_tracks, rows):
    from paper_2503_17608_amd import emstep
    t = np.zeros(len(orc_tracks), dtype=emstep.TRACK_DTYPE)
    t["key"] = orc_tracks["key"]
    t["row"] = rows
    t["step"] = orc_tracks["step"]
    t["type"] = orc_tracks["type"]
    t["slab"] = orc_tracks["slab"]
    t["T"] = orc_tracks["T"]
    t["nl"] = orc_tracks["nl"]
    t["r"] = orc_tracks["r"]
    t["u"] = orc_tracks["u"]
    return t


def layer_sums(edep):
    """Per-layer deposit (Pb + LAr pair of slabs)."""
    return edep.reshape(edep.shape[0], -1, 2).sum(2)


def ledger_int_mismatch(a, b, fields=("n_pair", "n_annih", "steps", "n_guard")):
    """Name of the first integer ledger field that differs between a and b, or None."""
    for f in fields:
        if not np.array_equal(a[f], b[f]):
            return f
    if not np.array_equal(a["n_sec"], b["n_sec"]):
        return "n_sec"
    return None


def run_oracle(w, events=None, threads=None):
    """Oracle per-event deposits, ledgers and total steps for the events of
    `w` (all, or the given ids in that order)."""
    import os
    pb = oracle.problem_for(w)
    if events is None:
        tr, rows = oracle.tracks_from_primaries(w.primaries)
        n = w.n_events
    else:
        events = np.asarray(events, dtype=np.uint64)
        p = w.primaries[np.isin(w.primaries["event"], events)]
        pos = {int(e): i for i, e in enumerate(events)}
        tr, rows = oracle.tracks_from_primaries(p, [pos[int(e)] for e in p["event"]])
        n = len(events)
    return pb.run_events(tr, rows, n, threads or len(os.sched_getaffinity(0)))


def event_energy(w):
    """Kinetic energy of every event's primaries."""
    return np.bincount(w.primaries["event"].astype(np.int64), weights=w.primaries["T"], minlength=w.n_events)


def flip_factory(w, msc=False):
    """Sessions for the flip diagnoser's step-by-step device histories."""
    def factory(n_slots):
        return session_for(w, n_slots=n_slots, max_events=1, sort_policy="none", graph_iterations=0,
                           max_substeps=0, msc=msc)
    return factory


def assert_events_match(w, edep, led, e_ref, l_ref, tag, events=None, msc=False, diagnose=True):
    """Device against the oracle, event by event: integer ledger equal and
    every per-slab deposit and the escaped energy within 1e-9 of the event's
    energy.  An event
    outside this is accepted only when the flip diagnoser finds the first
    discrete difference between its device and oracle histories (a different
    type, slab, interaction-length state, a track ending on one side only, or
    a per-step difference above 1e-6) at a step where the oracle's decision
    margin is no larger than the continuous per-step difference the two
    histories had already accumulated before it: rounding decided it.  At most
    0.1 % of the events (at least one) may be such flips."""
    e0 = event_energy(w)
    ev = np.arange(len(edep)) if events is None else np.asarray(events, dtype=np.int64)
    if events is not None:
        e0 = e0[ev]
    rel = np.maximum(np.abs(edep - e_ref).max(1), np.abs(led["escaped"] - l_ref["escaped"])) / e0
    int_bad = np.zeros(len(rel), dtype=bool)
    for f in ("n_pair", "n_annih", "steps", "n_guard"):
        int_bad |= led[f] != l_ref[f]
    int_bad |= np.any(led["n_sec"] != l_ref["n_sec"], axis=1)
    out = np.nonzero((rel > 1e-9) | int_bad)[0]
    print(tag, "max rel", rel.max(), "events beyond 1e-9 or with integer differences:", len(out))
    assert len(out) <= max(1, len(rel) // 1000), (tag, len(out), np.sort(rel)[-5:])
    if len(out) and not diagnose:
        raise AssertionError((tag, "events beyond 1e-9 where no diagnosis is run", ev[out], rel[out]))
    for i in out:
        d, f = fd.diagnose_event(w, int(ev[i]), flip_factory(w, msc), n_slots=16384, msc=msc)
        print(tag, "event", int(ev[i]), "rel", rel[i], "flip", f)
        assert f.index >= 0, (tag, int(ev[i]), "no discrete difference explains", rel[i], d)
        assert f.margin <= f.drift, (tag, int(ev[i]), f)


def assert_same_as(w, edep, led, edep0, led0, tag, events=None):
    """Two device runs of the same events (another policy, fill, fusion or
    drain setting): per-track arithmetic is identical, only the order of the
    FP64 tally additions differs, so integer ledgers are equal and deposits
    agree to 1e-12 of the event's energy."""
    e0 = event_energy(w)
    if events is not None:
        e0 = e0[np.asarray(events, dtype=np.int64)]
    bad = ledger_int_mismatch(led, led0)
    assert bad is None, (tag, bad)
    rel = np.abs(edep - edep0).max(1) / e0
    assert rel.max() <= 1e-12, (tag, rel.max())
    assert np.all(np.abs(led["escaped"] - led0["escaped"]) <= 1e-12 * e0), tag
