"""Deterministic appends as a race detector (paper, "Stepping algorithm":
vacancies are filled deterministically at the start of each iteration).

With `deterministic=True` the interaction kernels stage each track's
secondaries at its position in the interaction order and two kernels append
them in that order, so the initializer buffer -- and with it the slots the
fill assigns -- does not depend on which blocks reach the buffer first.  Two
runs of the same showers must then hold the same state after every
iteration: which slots are occupied, every field of every occupied slot and
every queued initializer, bit for bit, and the same live / queued counts.
A lost or misplaced update anywhere in the iteration shows up as a
difference.  Only the FP64 sums of the tallies may differ (their atomic
order), within 1e-12 of the event energy; the integer ledgers must be equal,
and the run must match the oracle."""
import numpy as np
import pytest

import workloads
from tests.gpu_helpers import event_energy, ledger_int_mismatch, run_oracle, session_for

pytestmark = pytest.mark.gpu


def _field_bits(t):
    """Per-field bytes of a structured array (padding excluded)."""
    return tuple(np.ascontiguousarray(t[name]).tobytes() for name in t.dtype.names)


def _slot_bits(t):
    """Which slots are occupied, and the fields of the occupied ones (a slot
    that was never written holds whatever the workspace held)."""
    occ = t["type"] >= 0
    return (occ.tobytes(),) + _field_bits(t[occ])


def _history(w, n_slots, precision, policy, fuse, streams):
    s = session_for(w, n_slots=n_slots, precision=precision, sort_policy=policy, graph_iterations=0,
                    streams=streams, deterministic=True, n_initializers=1 << 20)
    s.set_tuning(fuse_interactions=fuse)
    s.push(w.primaries)
    hist = []
    for _ in range(100000):
        c = s.step(1)
        hist.append((int(c["alive"]), int(c["queued"]), _slot_bits(s.read_tracks(n_slots)),
                     _field_bits(s.read_secondaries())))
        if c["alive"] == 0 and c["queued"] == 0 and c["pending_primaries"] == 0:
            break
    assert c["overflow"] == 0
    edep, led = s.tallies_by_event(np.arange(w.n_events))
    s.close()
    return hist, edep, led, int(c["steps"])


@pytest.mark.parametrize("precision,policy,fuse,streams", [("f64", "partition", True, 1),
                                                           ("f64", "none", False, 4),
                                                           ("mixed", "radix", True, 1)])
def test_two_runs_hold_identical_state_after_every_iteration(precision, policy, fuse, streams):
    # 1024 slots for 6 showers of 1 GeV: secondaries wait in the buffer for
    # most of the run, so the fill's choice among them is exercised
    w = workloads.electron_showers_1gev_field(6)
    n = 1024
    h0, e0, l0, steps0 = _history(w, n, precision, policy, fuse, streams)
    h1, e1, l1, steps1 = _history(w, n, precision, policy, fuse, streams)
    assert len(h0) == len(h1), (len(h0), len(h1))
    assert max(q for _, q, _, _ in h0) > 0          # the buffer held secondaries beyond the slots
    for it, (a, b) in enumerate(zip(h0, h1)):
        assert a[:2] == b[:2], (it, a[:2], b[:2])
        for name, x, y in zip(("slots", "initializers"), a[2:], b[2:]):
            assert x == y, (it, name, "differs between two runs")
    assert steps0 == steps1
    assert ledger_int_mismatch(l0, l1) is None
    e = event_energy(w)
    assert np.all(np.abs(e0 - e1).max(1) <= 1e-12 * e)
    if precision == "f64":
        e_ref, l_ref, steps = run_oracle(w)
        assert steps0 == steps
        assert ledger_int_mismatch(l0, l_ref) is None
        assert np.all(np.abs(e0 - e_ref).max(1) <= 1e-9 * e)


def test_deterministic_context_rejects_out_of_order_appends():
    from paper_2503_17608_amd import emstep
    w = workloads.electron_showers_1gev_field(1)
    s = session_for(w, n_slots=1024, sort_policy="partition", deterministic=True)
    with pytest.raises(emstep.EmsError):
        s.set_tuning(sort_policy="queue")
    with pytest.raises(emstep.EmsError):
        s.set_tuning(drain_threshold=4096)
    s.set_tuning(sort_policy="radix", fuse_interactions=True)     # in-order settings stay allowed
    s.close()
    with pytest.raises(emstep.EmsError):
        session_for(w, n_slots=1024, sort_policy="queue", deterministic=True)
