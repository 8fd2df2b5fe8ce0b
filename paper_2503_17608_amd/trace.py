"""Per-iteration trace of the step loop in Chrome trace-event JSON (opens in
Perfetto and chrome://tracing).

The paper studies how a run spends its time as the number of live tracks
falls (its analysis of the low-occupancy tail).  `record` steps a session
one iteration at a time with per-kernel HIP-event timing on, and keeps per
iteration: live / queued / pending tracks, steps completed, and the GPU time
of every kernel role.  `to_chrome_trace` turns the records into counter
tracks (occupancy, steps) and one slice per kernel role per iteration, laid
end to end on a GPU-time axis (the slices give each role's time, not the
overlap of concurrent streams).  `tail_analysis` bins the records by live
tracks and finds where the along-step time per track leaves its plateau
(the paper's analysis of along-step time against active tracks).

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


ALONG_ROLES = ("along_neutral", "along_charged", "along_field")


def tail_analysis(records, onset_factor=2.0):
    """The occupancy analysis of a recorded run: along-step GPU time per
    iteration and per live track, binned by live tracks (powers of two), and
    the tail onset: the largest live-track bin whose along-step time per
    track exceeds `onset_factor` times the lowest bin value (the plateau of
    a full device).  Also the share of the run's kernel time spent in the
    iterations below each bin."""
    rows = []
    for r in records:
        n = r["alive"]
        if n <= 0:
            continue
        along = sum(r["kernel_ms"].get(k, 0.0) for k in ALONG_ROLES)
        total = sum(r["kernel_ms"].values())
        rows.append((n, along, total, r["steps"]))
    if not rows:
        return {"bins": [], "onset_alive": None}
    total_ms = sum(x[2] for x in rows)
    bins = {}
    for n, along, total, steps in rows:
        b = n.bit_length() - 1
        e = bins.setdefault(b, [0, 0.0, 0.0, 0, 0])
        e[0] += 1
        e[1] += along
        e[2] += total
        e[3] += steps
        e[4] += n
    out = []
    for b in sorted(bins):
        it, along, total, steps, tracks = bins[b]
        out.append({"alive_from": 1 << b, "alive_to": (1 << (b + 1)) - 1, "iterations": it,
                    "along_us_per_iteration": 1e3 * along / it, "along_ns_per_track": 1e6 * along / tracks,
                    "kernel_us_per_iteration": 1e3 * total / it, "kernel_ns_per_step": 1e6 * total / max(steps, 1),
                    "share_of_kernel_time": total / total_ms})
    plateau = min(x["along_ns_per_track"] for x in out)
    onset = None
    for x in out:
        if x["along_ns_per_track"] > onset_factor * plateau:
            onset = x["alive_to"]
    below = 0.0
    for x in out:
        below += x["share_of_kernel_time"]
        x["share_at_or_below"] = below
    return {"bins": out, "plateau_along_ns_per_track": plateau, "onset_factor": onset_factor,
            "onset_alive": onset, "kernel_ms": total_ms}


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
