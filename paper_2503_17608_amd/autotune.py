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
   reordering and runs masked (the "per step phase" choice), timed end to end;
4. fused or per-process interaction kernels, and the drain threshold below
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


def autotune(session, sample, policies=("none", "partition", "radix", "queue"),
             thresholds=(0, 2048, 16384, 131072), blocks=BLOCK_CANDIDATES, repeats=1, cache=None, key=None,
             log=None, drains=(0, 16384, 65536)):
    """Tune `session` (an emstep.Session with geometry and tables loaded) on
    the primaries `sample`; applies and returns the chosen tuning."""
    if cache and key and os.path.exists(cache):
        db = json.load(open(cache))
        if key in db:
            t = db[key]
            session.set_tuning(sort_policy=t["sort_policy"], tail_threshold=t["tail_threshold"], block=t["block"],
                               fuse_interactions=t.get("fuse_interactions", False),
                               drain_threshold=t.get("drain_threshold", 0))
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
    # 4. interaction kernels fused or not, then the drain threshold
    fuse_t = {}
    for f in (False, True):
        session.set_tuning(fuse_interactions=f, drain_threshold=0)
        fuse_t[f] = min(_run(session, sample, events) for _ in range(repeats))
    best_fuse = min(fuse_t, key=fuse_t.get)
    drain_t = {}
    for dth in drains:
        session.set_tuning(fuse_interactions=best_fuse, drain_threshold=dth)
        drain_t[dth] = min(_run(session, sample, events) for _ in range(repeats))
    best_drain = min(drain_t, key=drain_t.get)
    say("fuse", fuse_t, "drain", drain_t)
    session.set_tuning(sort_policy=best_policy, tail_threshold=best_th, block=best_block,
                       fuse_interactions=best_fuse, drain_threshold=best_drain)
    result = {"sort_policy": best_policy, "tail_threshold": int(best_th), "block": best_block,
              "fuse_interactions": bool(best_fuse), "drain_threshold": int(best_drain),
              "policy_seconds": pol_t, "threshold_seconds": {str(k): v for k, v in th_t.items()},
              "fuse_seconds": {str(k): v for k, v in fuse_t.items()},
              "drain_seconds": {str(k): v for k, v in drain_t.items()},
              "block_ms": {r: {str(b): v for b, v in d.items()} for r, d in per_role.items()}}
    if cache and key:
        db = json.load(open(cache)) if os.path.exists(cache) else {}
        db[key] = result
        with open(cache, "w") as f:
            json.dump(db, f, indent=1)
    return result
