"""Slot counts that are neither a multiple of the four slots a vacancy thread
covers nor of a vacancy block's 4096: the ordered vacancy list, the list of
occupied slots (read by the listed walk of the along-steps and by the drain)
and the fill must stay exact at the ragged end of the slot array (paper,
"Stepping algorithm": vacancies are filled at the start of every
iteration).  A lost, doubled or misplaced slot changes the step count or the
integer ledgers against the oracle."""
import numpy as np
import pytest

import workloads
from tests.gpu_helpers import event_energy, ledger_int_mismatch, run_oracle, session_for

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("slots", [1001, 4097, 6143])
def test_ragged_slot_counts_match_oracle(slots):
    w = workloads.electron_showers_1gev_field(8, n_slots=slots)
    e_ref, l_ref, steps = run_oracle(w)
    e = event_energy(w)
    for drain in (0, 0xFFFFFFFF):
        s = session_for(w, n_slots=slots, sort_policy="partition", init_partition=True, n_initializers=1 << 20)
        s.set_tuning(drain_threshold=drain)
        s.push(w.primaries)
        c = s.run(max_iterations=200000)
        edep, led = s.tallies_by_event(np.arange(w.n_events))
        s.close()
        tag = (slots, drain)
        assert c["overflow"] == 0, tag
        assert c["steps"] == steps, (tag, c["steps"], steps)
        assert ledger_int_mismatch(led, l_ref) is None, (tag, ledger_int_mismatch(led, l_ref))
        assert np.all(np.abs(edep - e_ref).max(1) <= 1e-9 * e), tag
