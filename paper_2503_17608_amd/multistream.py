"""Event-parallel mode: several independent step loops on one GPU.

The paper compares two ways of feeding a GPU: one large track-slot array
stepping the tracks of many events together, and an event-parallel mode in
which every host thread owns a stream and its own (smaller) track arrays and
transports whole events on them.  Here each worker thread owns an
`emstep.Session` (its own stream, state arrays and tally rows); events are
handed out in chunks from a shared queue, so uneven showers balance across
the workers.  Every worker pushes its chunk, runs its loop until the slots
empty, reads the chunk's tallies and releases the rows.

Results per event do not depend on the mode (random numbers are keyed by
event and track), which the GPU tests check against the oracle.
"""
from __future__ import annotations

import threading
import time

import numpy as np

from .serving import split_events


def run_event_parallel(sessions, primaries, chunk_events=64, keep_results=True, chunk_log=None):
    """Transport `primaries` with one host thread per session.

    Returns (edep: {event: per-slab array}, ledger: {event: record}, steps, wall seconds).
    Each session needs max_events >= chunk_events.  With a list as
    `chunk_log`, one record per chunk is appended to it: the session, the
    chunk's start and end (seconds from the start of the call), the seconds
    spent in push, run and release, and its iterations and track-steps."""
    events = split_events(primaries)
    chunks = [events[i:i + chunk_events] for i in range(0, len(events), chunk_events)]
    lock = threading.Lock()
    next_chunk = [0]
    edep, ledger = {}, {}
    steps = [0] * len(sessions)
    errors = []

    def worker(k):
        s = sessions[k]
        prev = s.counters()
        c0 = prev["steps"]
        try:
            while True:
                with lock:
                    if next_chunk[0] >= len(chunks):
                        break
                    chunk = chunks[next_chunk[0]]
                    next_chunk[0] += 1
                ev = np.array([e for e, _ in chunk], dtype=np.uint64)
                ta = time.perf_counter()
                s.push(np.concatenate([p for _, p in chunk]))
                tb = time.perf_counter()
                c = s.run()
                tc = time.perf_counter()
                if keep_results:
                    e, led = s.tallies_by_event(ev)
                    for i, x in enumerate(ev):
                        edep[int(x)] = e[i]
                        ledger[int(x)] = led[i]
                s.release(ev)
                td = time.perf_counter()
                if chunk_log is not None:
                    with lock:
                        chunk_log.append({"session": k, "start": ta - t0, "end": td - t0, "push_s": tb - ta,
                                          "run_s": tc - tb, "release_s": td - tc, "iterations": int(c["iterations"] - prev["iterations"]),
                                          "steps": int(c["steps"] - prev["steps"])})
                prev = c
        except Exception as exc:          # surfaced to the caller below
            errors.append(exc)
        steps[k] = s.counters()["steps"] - c0

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(len(sessions))]
    t0 = time.perf_counter()
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    wall = time.perf_counter() - t0
    if errors:
        raise errors[0]
    return edep, ledger, sum(steps), wall
