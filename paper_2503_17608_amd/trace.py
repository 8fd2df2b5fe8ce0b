"""Per-iteration trace of the step loop in Chrome trace-event JSON (opens in
Perfetto and chrome://tracing).

The paper studies how a run spends its time as the number of live tracks
falls (its analysis of the low-occupancy tail).  `record` steps a session
one iteration at a time with per-kernel HIP-event timing on, and keeps per
iteration: live / queued / pending tracks, steps completed, and the GPU time
of every kernel role.  `to_chrome_trace` turns the records into counter
tracks (occupancy, steps) and one slice per kernel role per iteration, laid
end to end on a GPU-time axis (the slices give each role's time, not the
overlap of concurrent streams).

Command line:
    python -m paper_2503_17608_amd.trace --events 200 --out trace.json
"""
from __future__ import annotations

import argparse
import json

ROLE_ORDER = ("vacancies", "init", "sort", "along_neutral", "along_charged", "along_field", "compton",
              "photoelectric", "pair", "moller", "bhabha", "bremsstrahlung", "annihilation", "interactions", "drain")


def record(session, primaries, max_iterations=100_000):
    """Push `primaries` and step until the slots empty; one record per iteration."""
    from . import emstep
    session.push(primaries)
    session.profile(emstep.role_mask(*emstep.KERNEL_ROLES))
    session.profile_read()
    prev = session.counters()
    out = []
    try:
        for it in range(max_iterations):
            c = session.step(1)
            prof = session.profile_read()
            out.append({
                "iteration": it,
                "alive": int(c["alive"]), "queued": int(c["queued"]), "pending": int(c["pending_primaries"]),
                "steps": int(c["steps"] - prev["steps"]),
                "kernel_ms": {k: v[0] for k, v in prof.items() if v[1] > 0},
            })
            prev = c
            if c["alive"] == 0 and c["queued"] == 0 and c["pending_primaries"] == 0:
                break
    finally:
        session.profile(0)
    return out


def to_chrome_trace(records, name="step loop"):
    """Chrome trace-event document for `records` (as returned by `record`)."""
    ev = [{"name": "process_name", "ph": "M", "pid": 1, "args": {"name": name}},
          {"name": "thread_name", "ph": "M", "pid": 1, "tid": 1, "args": {"name": "kernels (GPU time)"}}]
    t = 0.0     # microseconds of summed GPU kernel time
    for r in records:
        ev.append({"name": "tracks", "ph": "C", "pid": 1, "ts": t,
                   "args": {"alive": r["alive"], "queued": r["queued"], "pending": r["pending"]}})
        ev.append({"name": "steps per iteration", "ph": "C", "pid": 1, "ts": t, "args": {"steps": r["steps"]}})
        t0 = t
        for role in ROLE_ORDER:
            ms = r["kernel_ms"].get(role)
            if not ms:
                continue
            dur = ms * 1e3
            ev.append({"name": role, "cat": "kernel", "ph": "X", "pid": 1, "tid": 1, "ts": t, "dur": dur,
                       "args": {"iteration": r["iteration"]}})
            t += dur
        ev.append({"name": f"iteration {r['iteration']}", "cat": "iteration", "ph": "X", "pid": 1, "tid": 2,
                   "ts": t0, "dur": t - t0, "args": {"alive": r["alive"], "steps": r["steps"]}})
    return {"traceEvents": ev, "displayTimeUnit": "ms"}


def write(records, path, name="step loop"):
    with open(path, "w") as f:
        json.dump(to_chrome_trace(records, name), f)


def main():
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads
    from . import emstep
    ap = argparse.ArgumentParser()
    ap.add_argument("--events", type=int, default=200)
    ap.add_argument("--slots", type=int, default=1 << 18)
    ap.add_argument("--policy", default="partition")
    ap.add_argument("--out", default="trace.json")
    a = ap.parse_args()
    w = workloads.electron_showers_1gev_field(a.events, n_slots=a.slots)
    st = w.stack
    s = emstep.Session(w.n_slots, max_events=w.n_events, max_slabs=st.n_slabs, max_materials=len(st.materials),
                       seed=w.seed, sort_policy=a.policy)
    s.load(st.z_planes, st.slab_material, st.half_width, st.B, st.materials, w.ecut)
    recs = record(s, w.primaries)
    s.close()
    write(recs, a.out, name=f"{w.name} {a.policy}")
    print(f"{len(recs)} iterations, {sum(r['steps'] for r in recs)} steps -> {a.out}")


if __name__ == "__main__":
    main()
