"""Per-iteration trace recorded from a real run: steps add up to the run's
total and the oracle's, occupancy ends at zero, every iteration has kernel
time."""
import numpy as np
import pytest

import workloads
from paper_2503_17608_amd import trace
from tests.gpu_helpers import run_oracle, session_for

pytestmark = pytest.mark.gpu


def test_recorded_trace_matches_run(tmp_path):
    w = workloads.electron_showers_1gev_field(10, n_slots=1 << 14)
    s = session_for(w, sort_policy="partition")
    recs = trace.record(s, w.primaries)
    c = s.counters()
    s.close()
    _, _, steps = run_oracle(w)
    assert sum(r["steps"] for r in recs) == c["steps"] == steps
    assert recs[-1]["alive"] == 0 and recs[-1]["queued"] == 0
    # every iteration but the last steps tracks (the pre-step runs in the along-step kernels)
    assert all(r["kernel_ms"].get("along_field", 0) + r["kernel_ms"].get("along_neutral", 0) > 0 for r in recs[:-1])
    p = tmp_path / "t.json"
    trace.write(recs, str(p))
    assert p.stat().st_size > 1000
    assert np.all(np.diff([r["iteration"] for r in recs]) == 1)
