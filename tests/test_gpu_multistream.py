"""Event-parallel mode: several sessions, each with its own stream, slot
arrays and host thread, transport chunks of events handed out from a shared
queue; every event's result equals the oracle's."""
import numpy as np
import pytest
import torch

import workloads
from paper_2503_17608_amd import multistream
from tests.gpu_helpers import ledger_int_mismatch, run_oracle, session_for

pytestmark = pytest.mark.gpu


def test_event_parallel_matches_oracle():
    w = workloads.electron_showers_1gev_field(24, n_slots=1 << 14)
    sessions = [session_for(w, n_slots=1 << 13, max_events=4, sort_policy=pol, graph_iterations=4, streams=1,
                            stream=torch.cuda.Stream())
                for pol in ("partition", "none", "queue")]
    edep, led, steps, wall = multistream.run_event_parallel(sessions, w.primaries, chunk_events=4)
    for s in sessions:
        s.close()
    e_ref, l_ref, steps_ref = run_oracle(w)
    assert steps == steps_ref
    assert sorted(edep) == list(range(w.n_events))
    e = np.stack([edep[i] for i in range(w.n_events)])
    lg = np.array([led[i] for i in range(w.n_events)], dtype=l_ref.dtype)
    assert ledger_int_mismatch(lg, l_ref) is None
    assert np.abs(e - e_ref).max() <= 1e-9 * 1000.0
