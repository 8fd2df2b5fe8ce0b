"""Pausing a field step at the substep cap is bit-transparent, track by track
(paper, "Reducing load imbalance": a capped propagation resumes in the next
iteration).

About 20 000 charged states in the 1 T stack are stepped once without a cap
(one iteration: along-step, then the interaction launch of the same
iteration), and in a second session with a cap of 1 or 3 RK4 evaluations per
iteration, one iteration at a time with no slot initialization, until each
track's step counter moves (or the track ends).  At that iteration the
capped track's state -- type, step, slab, T, n_lambda, position and
direction -- its event row's deposits, its ledger and the secondaries it
created must equal the uncapped ones bit for bit."""
import numpy as np
import pytest

import workloads
from tests.gpu_helpers import random_states, session_for, to_lib_tracks

pytestmark = pytest.mark.gpu

N = 20000


def _setup(w, states, precision, cap):
    s = session_for(w, n_slots=N, precision=precision, max_events=N, max_substeps=cap, n_initializers=16 * N)
    rows = np.array([s.register_event(int(e)) for e in states["event"]], dtype=np.uint32)
    s.inject(to_lib_tracks(states, rows))
    return s, rows


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint8)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
@pytest.mark.parametrize("cap", [1, 3])
def test_capped_field_step_is_bit_identical_per_track(precision, cap):
    w = workloads.electron_showers_1gev_field(1)
    rng = np.random.default_rng(101 + cap)
    states = random_states(w, N, rng, types=(1, 2), f32=precision == "mixed")
    # reference: one uncapped iteration
    ref, rows = _setup(w, states, precision, 0)
    ref.iterate(1, no_init=True)
    t_ref = ref.read_tracks(N)
    e_ref, l_ref, _ = ref.read_all()
    sec_ref = ref.read_secondaries()
    ref.close()
    # capped: one iteration at a time until every track's step has ended
    s, rows2 = _setup(w, states, precision, cap)
    assert np.array_equal(rows, rows2)
    done = np.zeros(N, dtype=bool)
    t_cap = np.zeros(N, dtype=t_ref.dtype)
    e_cap = np.zeros_like(e_ref)
    l_cap = np.zeros_like(l_ref)
    paused_seen = 0
    for it in range(4000):
        s.iterate(1, no_init=True)
        t = s.read_tracks(N)
        moved = ~done & ((t["type"] < 0) | (t["step"] != states["step"]))
        paused_seen += int(np.count_nonzero(~done & ~moved))
        for i in np.nonzero(moved)[0]:
            e, led = s.read_edep(int(states["event"][i]))
            e_cap[rows[i]] = e
            l_cap[rows[i]] = led
        t_cap[moved] = t[moved]
        done |= moved
        if done.all():
            break
    sec_cap = s.read_secondaries()
    c = s.counters()
    s.close()
    assert done.all(), f"{np.count_nonzero(~done)} steps still paused"
    assert paused_seen > 0 and c["work"]["field_paused"] > 0       # the cap really paused steps
    # every per-track field, bit for bit
    alive = t_ref["type"] >= 0
    assert np.array_equal(t_ref["type"], t_cap["type"])
    assert np.array_equal(t_ref["step"][alive], t_cap["step"][alive])
    for f in ("slab", "T", "nl", "r", "u"):
        assert np.array_equal(_bits(t_ref[f][alive]), _bits(t_cap[f][alive])), f
    # deposits and ledgers of every track's row, bit for bit
    assert np.array_equal(_bits(e_ref[rows]), _bits(e_cap[rows]))
    assert np.array_equal(_bits(l_ref[rows]), _bits(l_cap[rows]))
    # secondaries of the first step: each one of the reference (matched by
    # key) is in the capped session's buffer with identical values
    cap_by_key = {int(k): i for i, k in enumerate(sec_cap["key"])}
    assert len(sec_ref) > 100
    for r in sec_ref:
        j = cap_by_key.get(int(r["key"]))
        assert j is not None
        assert _bits(sec_cap[j:j + 1]).tobytes() == _bits(np.array([r])).tobytes()
