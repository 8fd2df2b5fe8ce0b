"""The autotuner on a small field workload (40 electrons of 1 GeV in the 1 T
stack at 2^16 slots): it picks block sizes, the sort policy, the tail
threshold, the phase table (reorder or mask per sort point and occupancy
bucket), fusion and the drain, applies them, and the tuned run still equals
the FP64 oracle event by event.  A phase table that masks each sort point in
half of the occupancy buckets gives the same results too."""
import numpy as np
import pytest

import workloads
from tests.gpu_helpers import assert_events_match, ledger_int_mismatch, run_oracle, session_for

pytestmark = pytest.mark.gpu


def _run(s, w):
    c0 = s.counters()["steps"]
    s.push(w.primaries)
    c = s.run(max_iterations=1_000_000)
    edep, led = s.tallies_by_event(np.arange(w.n_events))
    s.release(np.arange(w.n_events, dtype=np.uint64))
    return edep, led, c["steps"] - c0


def test_autotuned_run_matches_oracle():
    from paper_2503_17608_amd import autotune
    w = workloads.electron_showers_1gev_field(40, n_slots=1 << 16)
    e_ref, l_ref, steps = run_oracle(w)
    s = session_for(w, graph_iterations=8)
    res = autotune.autotune(s, w.primaries, blocks=(128, 256), thresholds=(0, 4096), drains=(0, 16384))
    t = s.tuning()
    assert tuple(t["phase_sort"]) == tuple(res["phase_sort"])
    assert t["drain_threshold"] == res["drain_threshold"] and t["fuse_interactions"] == res["fuse_interactions"]
    if res["sort_policy"] != "none":
        assert set(res["phase_table"]["choice"])            # the sample's buckets were timed
    edep, led, n = _run(s, w)
    assert n == steps
    assert_events_match(w, edep, led, e_ref, l_ref, "autotuned")
    # half the buckets masked at each sort point (complementary halves)
    s.set_tuning(sort_policy="partition", phase_sort=(0x0000FFFF, 0xFFFF0000), drain_threshold=0)
    edep2, led2, n2 = _run(s, w)
    s.close()
    assert n2 == steps
    assert ledger_int_mismatch(led2, led) is None
    assert np.all(np.abs(edep2 - edep) <= 1e-12 * w.primaries["T"][:, None])
