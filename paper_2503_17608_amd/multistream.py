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


def run_event_parallel(sessions, primaries, chunk_events=64, keep_results=True):
    """Transport `primaries` with one host thread per session.

    Returns (edep: {event: per-slab array}, ledger: {event: record}, steps, wall seconds).
    Each session needs max_events >= chunk_events."""
    events = split_events(primaries)
    chunks = [events[i:i + chunk_events] for i in range(0, len(events), chunk_events)]
    lock = threading.Lock()
    next_chunk = [0]
    edep, ledger = {}, {}
    steps = [0] * len(sessions)
    errors = []

    def worker(k):
        s = sessions[k]
        c0 = s.counters()["steps"]
        try:
            while True:
                with lock:
                    if next_chunk[0] >= len(chunks):
                        break
                    chunk = chunks[next_chunk[0]]
                    next_chunk[0] += 1
                ev = np.array([e for e, _ in chunk], dtype=np.uint64)
                s.push(np.concatenate([p for _, p in chunk]))
                s.run()
                if keep_results:
                    e, led = s.tallies_by_event(ev)
                    for i, x in enumerate(ev):
                        edep[int(x)] = e[i]
                        ledger[int(x)] = led[i]
                s.release(ev)
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
