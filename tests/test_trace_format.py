"""Chrome trace-event export of per-iteration records (host logic only)."""
import json

from paper_2503_17608_amd import trace


def _records():
    return [
        {"iteration": 0, "alive": 10, "queued": 4, "pending": 2, "steps": 10,
         "kernel_ms": {"sort": 0.01, "along_field": 0.05, "vacancies": 0.002}},
        {"iteration": 1, "alive": 3, "queued": 0, "pending": 0, "steps": 12,
         "kernel_ms": {"sort": 0.008, "compton": 0.004}},
    ]


def test_slices_are_laid_end_to_end_in_role_order():
    doc = trace.to_chrome_trace(_records())
    json.dumps(doc)                                   # serialisable
    ks = [e for e in doc["traceEvents"] if e.get("cat") == "kernel"]
    assert [e["name"] for e in ks] == ["vacancies", "sort", "along_field", "sort", "compton"]
    for a, b in zip(ks, ks[1:]):
        assert abs(a["ts"] + a["dur"] - b["ts"]) < 1e-9
    assert abs(sum(e["dur"] for e in ks) - 1e3 * (0.01 + 0.05 + 0.002 + 0.008 + 0.004)) < 1e-9
    its = [e for e in doc["traceEvents"] if e.get("cat") == "iteration"]
    assert [e["args"]["steps"] for e in its] == [10, 12]
    assert abs(its[1]["ts"] - (its[0]["ts"] + its[0]["dur"])) < 1e-9


def test_counter_tracks_carry_occupancy():
    doc = trace.to_chrome_trace(_records())
    cs = [e for e in doc["traceEvents"] if e["ph"] == "C" and e["name"] == "tracks"]
    assert [(c["args"]["alive"], c["args"]["queued"], c["args"]["pending"]) for c in cs] == [(10, 4, 2), (3, 0, 0)]
