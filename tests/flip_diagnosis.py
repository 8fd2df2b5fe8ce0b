"""Flip diagnosis: where and why a GPU event history leaves the oracle's.

The device loop and the oracle take the same decisions from inputs that
differ only by rounding (libm, FMA contraction, atomic order of tallies).  A
per-slab deposit that differs by more than rounding accumulates to must come
from a discrete decision taken the other way ("flip") where the oracle was
within rounding of the threshold.  This module finds the first step of an
event at which the two histories part and the oracle's decision margin
there:

* oracle side: ``Problem.trace_event`` records every step of the event in
  history order (ancestors first) with the smallest margin among the step's
  decisions (|a - b| / scale of each steering comparison) and its kind;
* device side: the event is run alone in a fresh session, one iteration at a
  time with no substep cap, no drain and no reordering, and every live
  track's state is read after every iteration; each iteration advances every
  live track by exactly one step, so the state after step k of track K is
  seen once;
* the first oracle record (in history order) whose post-step state the
  device does not reproduce to the per-step tolerance is the divergence; its
  track's earlier steps and the step that created the track all matched.

When the divergent step is a track's first step, the step that created the
track is reported as well, since a flip in the parent's sampling shows up
only in the child.  Test infrastructure: GPU tests only.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle


@dataclass
class Divergence:
    index: int                 # oracle record index (history order), -1 if none
    key: int
    step: int                  # pre-step counter of the divergent step
    what: str                  # which quantity differs
    rel_diff: float            # size of the difference (per-step metric)
    margin: float              # smallest oracle decision margin of the step
    kind: str                  # its decision kind
    parent_margin: float       # margin of the step that created the track (first steps only)
    parent_kind: str
    n_steps: int               # steps in the oracle history

    @property
    def flip_margin(self):
        m = self.margin
        if self.parent_margin == self.parent_margin:      # not NaN
            m = min(m, self.parent_margin)
        return m


def device_history(session_factory, prims, n_slots, max_iterations=200000):
    """States of every live track after every iteration of the event
    `prims` (library PRIMARY_DTYPE) run alone: structured array with the
    library's TRACK_DTYPE fields, one row per (key, step) reached alive."""
    s = session_factory(n_slots)
    s.push(prims)
    chunks = []
    for _ in range(max_iterations):
        c = s.step(1)
        t = s.read_tracks(n_slots)
        live = t[t["type"] >= 0]
        if len(live):
            chunks.append(live.copy())
        if len(live) == 0 and c["queued"] == 0 and c["pending_primaries"] == 0:
            break
    else:
        raise RuntimeError("event did not finish")
    s.close()
    return np.concatenate(chunks) if chunks else np.zeros(0, dtype=t.dtype)


def _state_diff(g, o, pre):
    """Per-step metric of one state (device record g, oracle post-step o,
    oracle pre-step pre): energies relative to the pre-step energy,
    directions absolute, positions relative to max(|r|, 1 cm), the
    interaction length relative to max(n_lambda, 1).  A different particle
    type, slab or interaction-length state is a discrete difference (inf)."""
    if int(g["type"]) != int(o["type"]) or int(g["slab"]) != int(o["slab"]):
        return "type/slab", np.inf
    T0 = max(abs(float(pre["T"])), 1e-300)
    d = {"T": abs(float(g["T"]) - float(o["T"])) / T0,
         "u": float(np.abs(g["u"] - o["u"]).max()),
         "r": float(np.abs(g["r"] - o["r"]).max() / max(np.linalg.norm(o["r"]), 1.0))}
    if (float(g["nl"]) < 0) != (float(o["nl"]) < 0):
        return "n_lambda set", np.inf
    if float(o["nl"]) >= 0:
        d["n_lambda"] = abs(float(g["nl"]) - float(o["nl"])) / max(abs(float(o["nl"])), 1.0)
    k = max(d, key=d.get)
    return k, d[k]


@dataclass
class Flip:
    index: int                 # oracle record index (history order) of the first discrete difference, -1 if none
    key: int
    step: int
    what: str
    margin: float              # smallest oracle decision margin of that step (or of the step that created the track)
    kind: str
    drift: float               # largest continuous per-step difference seen before it (any track)
    first_drift_index: int     # first record whose continuous difference exceeds the tolerance
    n_steps: int


def _compare(trace, dev, tol):
    at = {}
    for i in range(len(dev)):
        at[(int(dev["key"][i]), int(dev["step"][i]))] = i
    creator = {}
    for i in range(len(trace)):
        r = trace[i]["res"]
        for k in range(int(r["n_sec"])):
            creator[int(r["sec"][k]["key"])] = i
    for i in range(len(trace)):
        rec = trace[i]
        key, k1 = int(rec["post"]["key"]), int(rec["post"]["step"])
        j = at.get((key, k1))
        if rec["post"]["alive"]:
            if j is None:
                what, diff = "track ended on the device only", np.inf
            else:
                what, diff = _state_diff(dev[j], rec["post"], rec["pre"])
        elif j is not None:
            what, diff = "track ended in the oracle only", np.inf
        else:
            what, diff = "", 0.0
        yield i, rec, key, what, diff, creator


def first_divergence(trace, dev, tol=1e-12):
    """The first record (history order) whose post-step state the device does
    not reproduce to `tol`, with the oracle's decision margin there."""
    for i, rec, key, what, diff, creator in _compare(trace, dev, tol):
        if diff <= tol:
            continue
        pm, pk = float("nan"), ""
        if int(rec["pre"]["step"]) == 0 and key in creator:
            pr = trace[creator[key]]
            pm, pk = float(pr["m"]["margin"]), oracle.MARGIN_KINDS[int(pr["m"]["kind"])]
        return Divergence(i, key, int(rec["pre"]["step"]), what, float(diff), float(rec["m"]["margin"]),
                          oracle.MARGIN_KINDS[int(rec["m"]["kind"])], pm, pk, len(trace))
    return Divergence(-1, 0, 0, "", 0.0, np.inf, "", float("nan"), "", len(trace))


def first_flip(trace, dev, tol=1e-12):
    """The first discrete difference between the histories (a different
    particle type, slab, interaction-length state, a track that ends on one
    side only, or a per-step difference above 1e-6), with the oracle's decision margin at that step (the smaller of
    the step's and, for a track's first step, of the step that created it),
    and the largest continuous per-step difference seen before it."""
    drift, first_drift = 0.0, -1
    for i, rec, key, what, diff, creator in _compare(trace, dev, tol):
        # (a difference of 1e-6 in one step is no rounding drift in FP64:
        # the step took another process or sampled another final state)
        if np.isfinite(diff) and diff <= 1e-6:
            if diff > tol and first_drift < 0:
                first_drift = i
            drift = max(drift, diff)
            continue
        m, kind = float(rec["m"]["margin"]), oracle.MARGIN_KINDS[int(rec["m"]["kind"])]
        if int(rec["pre"]["step"]) == 0 and key in creator:
            pr = trace[creator[key]]
            if float(pr["m"]["margin"]) < m:
                m, kind = float(pr["m"]["margin"]), oracle.MARGIN_KINDS[int(pr["m"]["kind"])]
        return Flip(i, key, int(rec["pre"]["step"]), what, m, kind, drift, first_drift, len(trace))
    return Flip(-1, 0, 0, "", np.inf, "", drift, first_drift, len(trace))


def diagnose_event(w, event, session_factory, n_slots=8192, tol=1e-12, msc=False):
    """First continuous divergence and first discrete difference (flip) of
    event `event` of workload `w`, oracle against device."""
    prims = w.primaries[w.primaries["event"] == event]
    pb = oracle.problem_for(w, msc=msc)
    tr, _ = oracle.tracks_from_primaries(prims)
    trace = pb.trace_event(tr)
    dev = device_history(session_factory, prims, n_slots)
    return first_divergence(trace, dev, tol), first_flip(trace, dev, tol)
