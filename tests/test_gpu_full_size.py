"""GPU parity at the benchmark workloads' full sizes, in the launch
configuration the benchmark times (partition policy, charged / neutral
partitioned fill, 8-iteration graph batches, LDS-staged tables, one stream,
substep cap 10, photon and field along-steps in one launch, masked (no
sort point before them), fused interaction kernel, drain below 65536
tracks), plus degenerate and rejected inputs.

* 10^4 electrons of 1 GeV in the 1 T stack at 2^20 slots: every event of the
  benchmark's configuration against the FP64 oracle (integer ledger equal,
  deposits to 1e-9 of the primary energy, or a decision flip that the flip
  diagnoser shows rounding decided), and the sort policies none / radix /
  queue, the unpartitioned fill, parent-slot reuse, and the seven
  interaction kernels on four streams with no drain against that run
  (integer ledgers equal, deposits to 1e-12);
* 10^4 mixed primaries in a 5 degree cone at 2^20 slots: FP64 per event
  against the oracle, and the mixed-precision run's per-layer mean deposit
  within 0.5 % of the FP64 oracle;
* 64 events of 1-500 primaries up to 100 GeV at 2^22 slots: a sample of
  events computed by the oracle one by one (results of an event do not depend
  on what else is in flight), plus the exact energy ledger of every event;
* degenerate primaries (on a plane moving out, grazing, at the cut, low-energy
  positrons and photons) against the oracle; an empty push; invalid
  primaries rejected with nothing queued.
"""
import numpy as np
import pytest

import workloads
from tests.gpu_helpers import assert_events_match as _assert_events_match
from tests.gpu_helpers import assert_same_as as _assert_same_as
from tests.gpu_helpers import event_energy as _event_energy
from tests.gpu_helpers import layer_sums, run_oracle, session_for

pytestmark = pytest.mark.gpu

ME = 0.51099895
BENCH = dict(sort_policy="partition", init_partition=True, graph_iterations=8, lds_tables=1, streams=1,
             max_substeps=10)
BENCH_TUNING = dict(drain_threshold=65536, drain_steps=4096, fuse_interactions=True, fuse_along=True,
                    phase_sort=(0x0, 0xFFFFFFFF))


def _run(w, events=None, tuning=None, **kw):
    opts = dict(BENCH)
    opts.update(kw)
    s = session_for(w, **opts)
    t = dict(BENCH_TUNING)
    t.update(tuning or {})
    s.set_tuning(**t)
    s.push(w.primaries)
    c = s.run(max_iterations=1_000_000)
    ev = np.arange(w.n_events) if events is None else np.asarray(events)
    edep, led = s.tallies_by_event(ev)
    s.close()
    return edep, led, c


def _assert_ledger_exact(w, edep, led, events=None):
    e0 = _event_energy(w)
    if events is not None:
        e0 = e0[np.asarray(events, dtype=np.int64)]
    tot = edep.sum(1) + led["escaped"] + 2 * ME * (led["n_pair"].astype(float) - led["n_annih"])
    assert np.max(np.abs(tot - e0) / e0) < 1e-9


def test_full_size_electron_showers_every_policy():
    w = workloads.electron_showers_1gev_field()
    assert w.n_events == 10_000 and w.n_slots == 1 << 20
    e_ref, l_ref, steps = run_oracle(w)
    first = None
    for policy in ("partition", "none", "radix", "queue", "partition+fill0", "partition+reuse",
                   "partition+unfused+nodrain"):
        if policy == "partition+fill0":
            edep, led, c = _run(w, sort_policy="partition", init_partition=False)
        elif policy == "partition+reuse":
            edep, led, c = _run(w, sort_policy="partition", tuning=dict(reuse_parent_slot=True))
            assert c["work"]["reused_slots"] > 0 and c["work"]["drain"] > 0
        elif policy == "partition+unfused+nodrain":
            edep, led, c = _run(w, sort_policy="partition", streams=4,
                                tuning=dict(fuse_interactions=False, drain_threshold=0))
            assert c["work"]["drain"] == 0
        else:
            edep, led, c = _run(w, sort_policy=policy)
        assert c["overflow"] == 0, policy
        assert c["steps"] == steps, (policy, c["steps"], steps)
        if first is None:
            # the benchmark's configuration against the oracle ...
            _assert_events_match(w, edep, led, e_ref, l_ref, policy)
            first = (edep, led)
        else:
            # ... and every other configuration against it
            _assert_same_as(w, edep, led, first[0], first[1], policy)
    _assert_ledger_exact(w, edep, led)
    lg, lr = layer_sums(edep), layer_sums(e_ref)
    sig = np.sqrt(lg.var(0) / len(lg) + lr.var(0) / len(lr))
    assert np.all(np.abs(lg.mean(0) - lr.mean(0)) <= 3 * sig + 1e-12)


def test_full_size_mixed_cone_fp64_and_mixed_precision():
    w = workloads.mixed_cone_showers()
    assert w.n_events == 10_000 and w.n_slots == 1 << 20
    e_ref, l_ref, steps = run_oracle(w)
    edep, led, c = _run(w, precision="f64")
    assert c["steps"] == steps
    _assert_events_match(w, edep, led, e_ref, l_ref, "f64")
    _assert_ledger_exact(w, edep, led)
    edep_m, led_m, c_m = _run(w, precision="mixed")
    assert c_m["overflow"] == 0
    lg, lr = layer_sums(edep_m).mean(0), layer_sums(e_ref).mean(0)
    big = lr >= 0.01 * lr.sum()
    err = np.abs(lg[big] - lr[big]) / lr[big]
    print("mixed per-layer max rel err", err.max(), "layers", int(big.sum()))
    assert err.max() <= 0.005
    # FP32 energies still close the per-event ledger to FP32 resolution
    e0 = _event_energy(w)
    tot = edep_m.sum(1) + led_m["escaped"] + 2 * ME * (led_m["n_pair"].astype(float) - led_m["n_annih"])
    assert np.max(np.abs(tot - e0) / e0) < 1e-4


def test_full_size_batched_events_sampled():
    w = workloads.batched_mixed_events()
    assert w.n_events == 64 and w.n_slots == 1 << 22
    sample = np.array([0, 9, 17, 30, 41, 63])
    s = session_for(w, **BENCH)
    s.set_tuning(**BENCH_TUNING)
    s.push(w.primaries)
    c = s.run(max_iterations=1_000_000)
    edep_all, led_all = s.tallies_by_event(np.arange(w.n_events))
    s.close()
    assert c["overflow"] == 0
    _assert_ledger_exact(w, edep_all, led_all)
    e_ref, l_ref, _ = run_oracle(w, events=sample)
    # (events of up to 500 primaries of up to 100 GeV are too long for a
    # step-by-step diagnosis: here every sampled event must be within 1e-9)
    _assert_events_match(w, edep_all[sample], led_all[sample], e_ref, l_ref, "sample", events=sample,
                         diagnose=False)


def _degenerate_primaries(w):
    st = w.stack
    z = st.z_planes
    W = st.half_width
    rows = []
    # (type, T, r, u, slab)
    rows.append((1, 50.0, (0, 0, z[0]), (0, 0, -1.0), 0))                 # front face, moving out
    rows.append((0, 50.0, (0, 0, z[7]), (0, 0, -1.0), 7))                 # interior plane, moving back
    rows.append((2, 30.0, (0, 0, z[3]), (1.0, 0, 0), 3))                  # grazing along a plane
    rows.append((1, 20.0, (0.5, 0.5, 0.5 * (z[4] + z[5])), (0, 1.0, 0), 4))   # parallel to the planes
    rows.append((1, w.ecut * (1 + 1e-12), (0, 0, z[2] + 0.01), (0, 0, 1.0), 2))  # at the cut
    rows.append((2, w.ecut * 1.5, (0, 0, z[5] + 0.01), (0, 0, 1.0), 5))  # slow positron
    rows.append((0, max(1.5 * ME, 1.01 * w.ecut), (0, 0, z[1] + 0.01), (0, 0, 1.0), 1))  # below pair threshold
    rows.append((0, 2 * ME * (1 + 1e-9), (0, 0, z[1] + 0.01), (0, 0, 1.0), 1))  # just above it
    rows.append((1, 100.0, (W, -W, z[-1]), (0.0, 0.6, 0.8), st.n_slabs - 1))  # back corner, moving out
    rows.append((2, 200.0, (W * 0.999, 0, z[10] + 0.1), (1.0, 0, 0), 10))  # next to a lateral wall
    p = np.zeros(len(rows), dtype=workloads.PRIM_DTYPE)
    for i, (t, T, r, u, sl) in enumerate(rows):
        p[i]["event"] = i
        p[i]["key"] = 1000 + i
        p[i]["type"] = t
        p[i]["T"] = T
        p[i]["r"] = r
        p[i]["u"] = u
        p[i]["slab"] = sl
    return p


@pytest.mark.parametrize("field", [False, True])
def test_degenerate_primaries_match_oracle(field):
    base = workloads.electron_showers_1gev_field(1) if field else workloads.small_electron_showers(1)
    p = _degenerate_primaries(base)
    w = workloads.Workload(base.name + "_degenerate", base.stack, base.ecut, base.seed, len(p), p, 4096)
    e_ref, l_ref, steps = run_oracle(w)
    for policy in ("none", "partition"):
        edep, led, c = _run(w, sort_policy=policy)
        assert c["steps"] == steps, (policy, c["steps"], steps)
        _assert_events_match(w, edep, led, e_ref, l_ref, policy)
    _assert_ledger_exact(w, edep, led)


def test_empty_push_and_invalid_primaries_rejected():
    from paper_2503_17608_amd import emstep
    w = workloads.small_electron_showers(4)
    s = session_for(w, **BENCH)
    s.push(w.primaries[:0])
    c = s.run()
    assert c["steps"] == 0 and c["alive"] == 0 and c["queued"] == 0
    good = w.primaries[:1].copy()
    bad_cases = {}
    b = good.copy(); b["type"] = 5; bad_cases["type"] = b
    b = good.copy(); b["T"] = w.ecut * 0.5; bad_cases["below cut"] = b
    b = good.copy(); b["T"] = np.nan; bad_cases["nan energy"] = b
    b = good.copy(); b["u"] = (0.0, 0.0, 2.0); bad_cases["direction"] = b
    b = good.copy(); b["slab"] = w.stack.n_slabs; bad_cases["slab"] = b
    b = good.copy(); b["r"] = (0.0, 0.0, w.stack.z_planes[3]); bad_cases["z outside slab"] = b
    b = good.copy(); b["r"] = (2 * w.stack.half_width, 0.0, 0.0); bad_cases["outside wall"] = b
    for name, b in bad_cases.items():
        mixed = np.concatenate([w.primaries[1:3], b])      # valid ones first: nothing may be queued
        with pytest.raises(emstep.EmsError):
            s.push(mixed)
        c = s.counters()
        assert c["pending_primaries"] == 0, name
    s.push(w.primaries)
    c = s.run()
    e_ref, l_ref, steps = run_oracle(w)
    assert c["steps"] == steps
    edep, led = s.tallies_by_event(np.arange(w.n_events))
    _assert_events_match(w, edep, led, e_ref, l_ref, "after rejects")
    # a batch release with an unknown or a repeated id releases nothing
    for bad in ([0, 1, 999], [2, 2]):
        with pytest.raises(emstep.EmsError):
            s.release(np.array(bad, dtype=np.uint64))
    e2, _ = s.tallies_by_event(np.arange(w.n_events))
    assert np.array_equal(e2, edep)
    s.release(np.arange(w.n_events, dtype=np.uint64))
    _, _, rows = s.read_all()
    assert np.all(rows == np.uint64(2 ** 64 - 1))
    s.close()
