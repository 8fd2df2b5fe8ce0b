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


def test_tail_analysis_finds_where_time_per_track_leaves_its_plateau():
    # a device whose along-step time is max(latency floor, tracks x 1 ns):
    # 20 us floor, so below 20 000 tracks the time per track rises
    recs = []
    for i, n in enumerate([1 << 20, 700_000, 300_000, 100_000, 40_000, 15_000, 6_000, 2_000, 500, 100, 10]):
        along = max(0.020, n * 1e-6)                       # ms
        recs.append({"iteration": i, "alive": n, "queued": 0, "pending": 0, "steps": n,
                     "kernel_ms": {"along_field": along, "sort": 0.010}})
    a = trace.tail_analysis(recs, onset_factor=2.0)
    assert abs(a["plateau_along_ns_per_track"] - 1.0) < 1e-9
    # 15 000 tracks (bin 8192-16383) cost 1.33 ns per track, 6 000 tracks
    # (bin 4096-8191) 3.3 ns: the tail starts in the 4096-8191 bin
    assert a["onset_alive"] == 8191
    assert abs(a["bins"][-1]["share_at_or_below"] - 1.0) < 1e-12
    assert sum(b["iterations"] for b in a["bins"]) == len(recs)
    top = a["bins"][-1]
    assert top["alive_from"] == 1 << 20 and abs(top["along_ns_per_track"] - 1.0) < 1e-9
