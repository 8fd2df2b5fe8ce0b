"""Autotuner for the step loop: sort policy, tail threshold, block sizes.

The knobs change speed only -- the physics results do not depend on them
(random numbers are keyed by track, not by slot or launch shape) -- so the
tuner may try them on the real workload, or on a sample that fills the slots
as the real workload does (a small fraction of the events does not: at low
occupancy masked stepping and no drain look best):

1. block sizes: the sample runs once per candidate block size with every
   step kernel at that size and per-kernel HIP-event timing on; each kernel
   role then keeps the size that minimised its own total time;
2. sort policy: none / partition / radix / queue, timed end to end;
3. tail threshold: the live-track count below which an iteration skips the
   reordering and runs masked, timed end to end;
4. the phase table: for each sort point (before the along-step kernels,
   before the interaction kernels) and each occupancy bucket floor(log2 live
   tracks), reorder or run masked.  The sample is stepped one iteration at a
   time with per-kernel HIP-event timing in the four combinations (both sort
   points reordering, either one, neither); the live-track count of every
   iteration is the same in all four (each track takes one step per
   iteration whatever the launch shape), so each bucket keeps the
   combination whose iterations in that bucket took the least GPU time;
5. fused or per-process interaction kernels, and the drain threshold below
   which the last tracks are drained in block-local loops, timed end to end.

Results can be cached in a JSON file keyed by a workload signature.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import emstep

BLOCK_CANDIDATES = (64, 128, 256, 512)
STEP_ROLES = ("along_neutral", "along_charged", "along_field", "compton", "photoelectric", "pair",
              "moller", "bhabha", "bremsstrahlung", "annihilation", "interactions")


def signature(n_slots, precision, stack, ecut, primaries):
    h = hashlib.sha1()
    h.update(json.dumps([int(n_slots), precision, float(ecut), list(map(float, stack.z_planes)),
                         list(map(int, stack.slab_material)), float(stack.half_width), list(stack.B),
                         [list(m) for m in stack.materials]]).encode())
    h.update(np.ascontiguousarray(primaries).tobytes())
    return h.hexdigest()[:16]


def _run(session, primaries, events):
    import torch
    session.push(primaries)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    session.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    session.release(events)
    return dt


ALL_BUCKETS = 0xFFFFFFFF


def iteration_times(session, primaries, events, max_iterations=200_000):
    """Step `primaries` one iteration at a time with per-kernel HIP-event
    timing: (live tracks, summed kernel ms) of every iteration, and the
    track-steps the run took."""
    session.push(primaries)
    session.profile(emstep.role_mask(*emstep.KERNEL_ROLES))
    session.profile_read()
    out = []
    steps0 = int(session.counters().get("steps", 0)) if hasattr(session, "counters") else None
    steps = None
    try:
        for _ in range(max_iterations):
            c = session.step(1)
            prof = session.profile_read()
            out.append((int(c["alive"]), sum(v[0] for v in prof.values() if v[1] > 0)))
            if steps0 is None:
                steps0 = int(c.get("steps", 0))
            steps = int(c.get("steps", 0))
            if c["alive"] == 0 and c["queued"] == 0 and c["pending_primaries"] == 0:
                break
    finally:
        session.profile(0)
    session.release(events)
    return out, (steps or 0) - (steps0 or 0)


def phase_table(session, sample, events):
    """Per sort point and occupancy bucket: reorder or run masked (step 4 of
    the module docstring).  Returns the two bucket masks and, per bucket, the
    kernel time per live track of the four combinations.

    Once the initializer queue holds more tracks than there are vacancies,
    which of them take the free slots follows the order in which the
    interactions appended them, and that order follows the slot order the
    sort points produce: the live-track count of an iteration can differ
    between the combinations while every track's history, and so the run's
    total of track-steps, is the same.  Buckets are therefore compared by
    kernel time per live track."""
    combos = {(1, 1): (ALL_BUCKETS, ALL_BUCKETS), (0, 1): (0, ALL_BUCKETS), (1, 0): (ALL_BUCKETS, 0), (0, 0): (0, 0)}
    per = {}
    steps_ref = None
    for combo, masks in combos.items():
        session.set_tuning(phase_sort=masks)
        rec, steps = iteration_times(session, sample, events)
        if steps_ref is None:
            steps_ref = steps
        elif steps != steps_ref:
            raise RuntimeError(f"track-steps differ between launch shapes ({steps} against {steps_ref})")
        ms, tracks = {}, {}
        for a, t in rec:
            if a > 0:
                b = a.bit_length() - 1
                ms[b] = ms.get(b, 0.0) + t
                tracks[b] = tracks.get(b, 0) + a
        per[combo] = {b: ms[b] / tracks[b] for b in ms}
    m1 = m2 = 0
    buckets = sorted(set().union(*[set(t) for t in per.values()]))
    choice = {}
    for b in buckets:
        best = min(combos, key=lambda k: per[k].get(b, float("inf")))
        choice[b] = best
        m1 |= best[0] << b
        m2 |= best[1] << b
    # buckets the sample never reached keep reordering
    seen = sum(1 << b for b in buckets)
    m1 |= ALL_BUCKETS & ~seen
    m2 |= ALL_BUCKETS & ~seen
    return (m1, m2), {"choice": {str(b): list(c) for b, c in choice.items()},
                      "ms_per_track": {f"{k[0]}{k[1]}": {str(b): v for b, v in t.items()} for k, t in per.items()}}


def autotune(session, sample, policies=("none", "partition", "radix", "queue"),
             thresholds=(0, 2048, 16384, 131072), blocks=BLOCK_CANDIDATES, repeats=1, cache=None, key=None,
             log=None, drains=(0, 16384, 65536), phases=True):
    """Tune `session` (an emstep.Session with geometry and tables loaded) on
    the primaries `sample`; applies and returns the chosen tuning."""
    if cache and key and os.path.exists(cache):
        db = json.load(open(cache))
        if key in db:
            t = db[key]
            session.set_tuning(sort_policy=t["sort_policy"], tail_threshold=t["tail_threshold"], block=t["block"],
                               fuse_interactions=t.get("fuse_interactions", False),
                               drain_threshold=t.get("drain_threshold", 0), fuse_along=t.get("fuse_along", True),
                               phase_sort=t.get("phase_sort", (ALL_BUCKETS, ALL_BUCKETS)))
            return t
    events = np.unique(sample["event"])
    say = log or (lambda *a: None)
    _run(session, sample, events)          # warm-up (graph capture, caches)
    # 1. per-kernel block sizes
    per_role = {r: {} for r in STEP_ROLES}
    mask = emstep.role_mask(*STEP_ROLES)
    for b in blocks:
        session.set_tuning(block={r: b for r in STEP_ROLES})
        session.profile(mask)
        session.profile_read()
        for _ in range(repeats):
            _run(session, sample, events)
        prof = session.profile_read()
        session.profile(0)
        for r in STEP_ROLES:
            ms, n = prof.get(r, (0.0, 0))
            if n:
                per_role[r][b] = ms
    best_block = {r: min(v, key=v.get) for r, v in per_role.items() if v}
    session.set_tuning(block=best_block)
    say("block sizes", best_block)
    # 2. sort policy
    pol_t = {}
    for p in policies:
        session.set_tuning(sort_policy=p, tail_threshold=0)
        pol_t[p] = min(_run(session, sample, events) for _ in range(repeats))
    best_policy = min(pol_t, key=pol_t.get)
    say("policies", pol_t)
    # 3. tail threshold for the chosen policy
    th_t = {}
    if best_policy != "none":
        for th in thresholds:
            session.set_tuning(sort_policy=best_policy, tail_threshold=th)
            th_t[th] = min(_run(session, sample, events) for _ in range(repeats))
        best_th = min(th_t, key=th_t.get)
    else:
        best_th = 0
    say("thresholds", th_t)
    session.set_tuning(sort_policy=best_policy, tail_threshold=best_th, block=best_block)
    # 4. phase table (per sort point and occupancy bucket), drain off so that
    # every iteration of the sample is a step-loop iteration
    phase_masks, phase_info = (ALL_BUCKETS, ALL_BUCKETS), {}
    if phases and best_policy != "none":
        session.set_tuning(drain_threshold=0)
        phase_masks, phase_info = phase_table(session, sample, events)
        say("phase table", phase_info.get("choice"))
        # the table decides per bucket, but a sort point skipped in every
        # bucket is not launched at all, which no bucket's time shows: try
        # each point off entirely against the table
        cand = {"table": phase_masks, "no point 1": (0, phase_masks[1]), "no point 2": (phase_masks[0], 0)}
        cand_t = {}
        for name, masks in cand.items():
            session.set_tuning(phase_sort=masks)
            cand_t[name] = min(_run(session, sample, events) for _ in range(repeats))
        phase_masks = cand[min(cand_t, key=cand_t.get)]
        phase_info["whole_point_seconds"] = cand_t
        say("phase table against whole sort points off", cand_t)
    session.set_tuning(phase_sort=phase_masks)
    # 5. interaction kernels fused or not, the along-steps fused or not, then
    # the drain threshold
    fuse_t = {}
    for f in (False, True):
        session.set_tuning(fuse_interactions=f, drain_threshold=0)
        fuse_t[f] = min(_run(session, sample, events) for _ in range(repeats))
    best_fuse = min(fuse_t, key=fuse_t.get)
    along_t = {}
    for f in (False, True):
        session.set_tuning(fuse_interactions=best_fuse, fuse_along=f, drain_threshold=0)
        along_t[f] = min(_run(session, sample, events) for _ in range(repeats))
    best_along = min(along_t, key=along_t.get)
    drain_t = {}
    for dth in drains:
        session.set_tuning(fuse_interactions=best_fuse, fuse_along=best_along, drain_threshold=dth)
        drain_t[dth] = min(_run(session, sample, events) for _ in range(repeats))
    best_drain = min(drain_t, key=drain_t.get)
    say("fuse", fuse_t, "fuse along", along_t, "drain", drain_t)
    session.set_tuning(sort_policy=best_policy, tail_threshold=best_th, block=best_block,
                       fuse_interactions=best_fuse, fuse_along=best_along, drain_threshold=best_drain,
                       phase_sort=phase_masks)
    result = {"sort_policy": best_policy, "tail_threshold": int(best_th), "block": best_block,
              "fuse_interactions": bool(best_fuse), "fuse_along": bool(best_along), "drain_threshold": int(best_drain),
              "phase_sort": [int(phase_masks[0]), int(phase_masks[1])], "phase_table": phase_info,
              "policy_seconds": pol_t, "threshold_seconds": {str(k): v for k, v in th_t.items()},
              "fuse_seconds": {str(k): v for k, v in fuse_t.items()},
              "fuse_along_seconds": {str(k): v for k, v in along_t.items()},
              "drain_seconds": {str(k): v for k, v in drain_t.items()},
              "block_ms": {r: {str(b): v for b, v in d.items()} for r, d in per_role.items()}}
    if cache and key:
        db = json.load(open(cache)) if os.path.exists(cache) else {}
        db[key] = result
        with open(cache, "w") as f:
            json.dump(db, f, indent=1)
    return result
