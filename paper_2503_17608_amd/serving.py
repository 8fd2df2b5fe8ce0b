"""Continuous-batching serving loop over the step-loop library.

Requests are events (showers of uneven size) arriving over time.  An arrived
event is admitted as soon as the device has room -- a free tally row and
enough headroom under the track budget (live tracks + queued secondaries +
pending primaries) -- and its primaries join the tracks already stepping on
the device: nothing waits for a batch to drain.  The host enqueues a fixed
number of step iterations (replayed HIP graphs when the session was created
with graph batches), then polls the device completion ring; every completed
event's tallies are read back and its row released for the next admission.

Latency of an event = time its completion was observed by the host - its
arrival time (host monotonic clock).  All stepping, tallying and completion
detection runs in the library's kernels; this module only schedules.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ServeResult:
    latency_s: dict = field(default_factory=dict)       # event id -> seconds
    edep: dict = field(default_factory=dict)            # event id -> per-slab deposit
    ledger: dict = field(default_factory=dict)
    wall_s: float = 0.0
    steps: int = 0
    iterations: int = 0
    max_in_flight: int = 0

    def percentile(self, q):
        v = np.sort(np.array(list(self.latency_s.values())))
        if len(v) == 0:
            return float("nan")
        k = int(np.ceil(q / 100.0 * len(v))) - 1      # nearest rank
        return float(v[min(max(k, 0), len(v) - 1)])


def split_events(primaries):
    """Primaries (PRIMARY_DTYPE-like) grouped by event id, in first-seen order."""
    order = collections.OrderedDict()
    for i, e in enumerate(primaries["event"]):
        order.setdefault(int(e), []).append(i)
    return [(e, primaries[np.array(idx)]) for e, idx in order.items()]


def serve(session, events, arrivals, track_budget, iterations_per_poll=8, keep_results=True,
          clock=time.perf_counter):
    """Run the serving loop until every event has completed.

    events:   list of (event id, primaries array) in arrival order
    arrivals: arrival time of each event [s], relative to the start
    track_budget: admit while live + queued + pending stays below this
    """
    res = ServeResult()
    waiting = collections.deque(range(len(events)))
    in_flight = {}
    free_rows = session.options.max_events
    c0 = session.counters()
    load = 0
    t0 = clock()
    while waiting or in_flight:
        now = clock() - t0
        # admission: arrived events, while rows and the track budget allow
        admitted = False
        while waiting and arrivals[waiting[0]] <= now and free_rows > 0 and load < track_budget:
            k = waiting.popleft()
            ev, prims = events[k]
            session.push(prims)
            in_flight[ev] = arrivals[k]
            free_rows -= 1
            load += len(prims)
            admitted = True
        res.max_in_flight = max(res.max_in_flight, len(in_flight))
        if not in_flight:
            # idle until the next arrival
            if waiting:
                dt = arrivals[waiting[0]] - (clock() - t0)
                if dt > 0:
                    time.sleep(min(dt, 0.01))
            continue
        session.launch(iterations_per_poll)
        done = session.poll_completed()
        t_done = clock() - t0
        for ev in done:
            ev = int(ev)
            res.latency_s[ev] = t_done - in_flight.pop(ev)
            if keep_results:
                e, led = session.read_edep(ev)
                res.edep[ev] = e
                res.ledger[ev] = led
            session.release(ev)
            free_rows += 1
        c = session.last_counters()          # the poll's snapshot: no second synchronization
        if c["overflow"]:
            # dropped secondaries: results of events in flight are incomplete
            raise RuntimeError("initializer buffer overflow while serving: increase n_initializers")
        load = c["alive"] + c["queued"] + c["pending_primaries"]
        del admitted
    res.wall_s = clock() - t0
    c1 = session.counters()
    res.steps = c1["steps"] - c0["steps"]
    res.iterations = c1["iterations"] - c0["iterations"]
    return res
