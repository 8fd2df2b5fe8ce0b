"""Benchmark: track-steps/s of the step-based EM shower loop on one MI355X.

One benchmark step is one pass of the whole hot path over one batch: every
primary of the workload transported until no track is alive, queued or
pending (vacancy compaction, initialization, pre-step, sort, along-step,
interactions, tallies).  Primaries are copied to the device before the timed
region of each step; `value` times the device loop only (inputs resident in
HBM), and `io_inclusive` times push + loop + readback of every tally.

Default workload: 10^4 electrons of 1 GeV into a 50-layer Pb (2 mm) / liquid
Ar (5 mm) stack, 40 x 40 cm, uniform 1 T field along x, 0.1 MeV cut, 2^20
track slots, FP64, slots sorted by next action, iterations replayed from
captured HIP graphs, the interaction kernels fused into one launch, the
last tracks (below 65536 alive, queued or pending) stepped in block-local loops by
the drain kernel.

The JSON line carries the dominant kernel's roofline: algorithmic bytes per
launch (the kernel's units of work times the bytes per unit fixed from the
state's field widths) divided by its average launch duration, measured with
HIP start/stop events stamped by the kernel's own dispatch packets in one
extra pass over the same batch (graph replay off for that pass); `traffic`
is the calibrated hardware byte count per launch from a committed counter
summary, when one was taken on the current kernel sources and this
configuration; and the oracle's throughput on the host cores for a bounded
sample of the same events.

The rest of the metric comes in the same line (skip with --no-extras):
`unsorted` (the same run with sort policy none), `precision_pair` (mixed
precision against FP64 on 10^4 mixed-species primaries in a 5 degree cone,
with the mixed run's per-layer error against the FP64 oracle) and `serving`
(continuous batching of 1000 events of 1-200 primaries at Poisson arrival
rates 0.5 / 0.7 / 0.9 x the sustained event rate of the closed FP64 batch of
the same events, p50/p99 latency in mixed precision and FP64, and the mixed
serving run's per-layer error against the FP64 oracle on a subsample).

Other modes: --autotune (tune policy / tail threshold / block sizes /
fusion / drain on the workload first), --layer-error (per-layer deposit of
this run against the FP64 oracle on the same events), --serve (the serving
section alone), --fig2 (along-step time per live track against live tracks,
and what the drain of the last tracks recovers), --sweep (throughput against
total track slots, mixed-event and event-parallel modes).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per unit of work, fixed before any measurement from the
# per-slot field widths of the state (FP64 / mixed): the fields a track that
# takes an action reads and writes, independent of how a kernel moves them.
#   pre-step 53 / 41, neutral along-step 110 / 86, charged along-step
#   134 / 106, field along-step 174 / 134 per completed step and 112 / 100 per
#   paused trip, deposit 16 (tally read-modify-write), interaction 116 / 84,
#   secondary 71 / 59 (initializer record written by the interaction) and
#   172 / 140 when it is initialized (record read, state written), post-step
#   19 / 15 per completed along-step.
# The along-step kernels run the pre-step of their tracks (a resumed field
# step has none) and fold the post-step in; the charged ones deposit.
UNIT_BYTES = {
    "f64": {"pre": 53, "neutral": 110, "charged": 134, "field": 174, "pause": 112, "deposit": 16,
            "interaction": 116, "secondary": 71, "init": 172, "post": 19},
    "mixed": {"pre": 41, "neutral": 86, "charged": 106, "field": 134, "pause": 100, "deposit": 16,
              "interaction": 84, "secondary": 59, "init": 140, "post": 15},
}
INTERACTIONS = ("compton", "photoelectric", "pair", "moller", "bhabha", "bremsstrahlung", "annihilation")


def kernel_bytes(kernel, work, precision):
    """Algorithmic bytes of `kernel` for the work counters `work` (tracks
    processed per role, paused field trips)."""
    u = UNIT_BYTES[precision]
    if kernel == "along_field":
        trips, paused = work.get("along_field", 0), work.get("field_paused", 0)
        done = trips - paused
        # every trip that is not a resumption runs the pre-step; in the
        # steady state resumptions equal the pauses of the launch before
        return done * (u["field"] + u["pre"] + u["deposit"] + u["post"]) + paused * u["pause"]
    if kernel == "along_neutral":
        return work.get("along_neutral", 0) * (u["neutral"] + u["pre"] + u["post"])
    if kernel == "along_charged":
        return work.get("along_charged", 0) * (u["charged"] + u["pre"] + u["deposit"] + u["post"])
    if kernel == "interactions":
        return sum(work.get(k, 0) for k in INTERACTIONS) * u["interaction"]
    if kernel == "init":
        return work.get("init", 0) * u["init"]
    if kernel == "drain":
        # a drain trip counts as a field step with its pre-step (its
        # interactions and secondaries are not counted)
        return work.get("drain", 0) * (u["field"] + u["pre"] + u["deposit"] + u["post"])
    raise KeyError(kernel)


PROFILES = os.path.join(ROOT, "profiles")


def source_digest():
    """SHA-256 over the library's kernel and ABI sources: hardware byte counts
    taken on other sources do not describe the current kernels."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2503_17608_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hpp", ".hip")))
    files.append(os.path.join(ROOT, "include", "emstep.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def committed_traffic(kernel, key):
    """Calibrated HBM bytes per launch of `kernel` from a committed counter
    summary (a `traffic:` JSON line in profiles/*.md) taken on these exact
    sources and this configuration; None when there is none."""
    if not os.path.isdir(PROFILES):
        return None
    digest = source_digest()
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith(".md"):
            continue
        for line in open(os.path.join(PROFILES, name)):
            if not line.startswith("traffic: "):
                continue
            try:
                t = json.loads(line[len("traffic: "):])
            except ValueError:
                continue
            if t.get("kernel") == kernel and t.get("sources_sha256") == digest and t.get("config") == key:
                return t
    return None


WORKLOADS = ("electron_showers_1gev_field", "small_electron_showers", "mixed_cone_showers",
             "batched_mixed_events", "serving_events", "lhc_like_events")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="electron_showers_1gev_field", choices=WORKLOADS)
    ap.add_argument("--events", type=int, default=0, help="override the number of events")
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--precision", default="", choices=["", "f64", "mixed"])
    ap.add_argument("--policy", default="partition", choices=["none", "partition", "radix", "queue"])
    ap.add_argument("--init-partition", type=int, default=1)
    ap.add_argument("--max-substeps", type=int, default=10)
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--graph", type=int, default=8, help="iterations per captured HIP graph (0 = plain launches)")
    ap.add_argument("--lds-tables", type=int, default=1)
    ap.add_argument("--streams", type=int, default=1)
    ap.add_argument("--drain-threshold", type=int, default=65536,
                    help="drain the last tracks in block-local loops below this many live+queued+pending (0 = off)")
    ap.add_argument("--drain-steps", type=int, default=4096,
                    help="drain rounds per launch (each of up to 4 steps per track)")
    ap.add_argument("--reuse-parent-slot", type=int, default=0, help="a finished track hands its slot to a secondary")
    ap.add_argument("--fuse-interactions", type=int, default=1, help="one launch for the seven interaction kernels")
    ap.add_argument("--phase-sort", type=lambda x: int(x, 0), nargs=2, default=[0x0, 0xFFFFFFFF],
                    metavar=("MASK1", "MASK2"),
                    help="reorder at sort point 1 / 2 in the occupancy buckets floor(log2 live tracks) whose bits "
                         "are set (an empty mask: that point's kernels are not launched); default: no sort point 1 "
                         "(the partitioned fill keeps photons and charged tracks apart and the along-step launch "
                         "runs masked), sort point 2 always")
    ap.add_argument("--fuse-along", type=int, default=1,
                    help="one launch for the photon and field along-steps (with a field and one stream)")
    ap.add_argument("--roofline-kernel", default="along_field")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--cpu-events", type=int, default=10000, help="oracle sample (events); 0 = skip")
    ap.add_argument("--compare", action="store_true", help="also time the other sort policies")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--layer-error", action="store_true")
    ap.add_argument("--serve", action="store_true")
    ap.add_argument("--serve-events", type=int, default=1000)
    ap.add_argument("--load", type=float, default=0.7, help="arrival rate / closed-batch event rate")
    ap.add_argument("--extra-loads", type=float, nargs="*", default=[0.5, 0.9],
                    help="further loads served (same arrival seed) after the main one")
    ap.add_argument("--serve-sample-every", type=int, default=20,
                    help="per-layer error of the mixed-precision serving run on every n-th event (0 = skip)")
    ap.add_argument("--no-extras", action="store_true",
                    help="the main workload only: no unsorted rate, precision pair or serving section")
    ap.add_argument("--fig2", action="store_true",
                    help="occupancy analysis: along-step time per live track against live tracks, and what the "
                         "drain recovers")
    ap.add_argument("--trace-out", default="", help="with --fig2: write the Chrome trace of the recorded run here")
    ap.add_argument("--sweep", action="store_true",
                    help="throughput against total track slots (2^14..2^23), mixed-event and event-parallel")
    ap.add_argument("--sweep-exp", type=int, nargs=2, default=[14, 23], help="slot exponents of the sweep")
    ap.add_argument("--sweep-k", type=int, nargs="*", default=[2, 4, 8], help="event-parallel session counts")
    ap.add_argument("--initializers", type=int, default=0,
                    help="initializer records of the mixed-event session in the sweep, shared out among the "
                         "event-parallel sessions (0 = max(16 x slots, 2^24))")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the run, copy a device buffer of this size three times (a reference kernel "
                         "of known traffic for hardware byte counters)")
    return ap.parse_args()


def make_workload(name, events, slots):
    import workloads
    kw = {}
    if events:
        kw["n_events"] = events
    w = getattr(workloads, name)(**kw)
    if slots:
        w.n_slots = slots
    return w


def new_session(w, args, precision, policy, init_partition, graph=None, drain=None, reuse=None, fuse=None,
                n_initializers=None):
    from paper_2503_17608_amd import emstep
    st = w.stack
    s = emstep.Session(w.n_slots, precision=precision, max_events=max(w.n_events, 1), max_slabs=st.n_slabs,
                       n_initializers=n_initializers,
                       max_materials=len(st.materials), seed=w.seed, sort_policy=policy,
                       init_partition=init_partition, max_substeps=args.max_substeps, block_size=args.block_size,
                       graph_iterations=args.graph if graph is None else graph, lds_tables=args.lds_tables,
                       streams=args.streams, n_primaries=max(len(w.primaries), 1 << 16))
    s.load(st.z_planes, st.slab_material, st.half_width, st.B, st.materials, w.ecut)
    drain = args.drain_threshold if drain is None else drain
    reuse = args.reuse_parent_slot if reuse is None else reuse
    fuse = args.fuse_interactions if fuse is None else fuse
    s.set_tuning(drain_threshold=drain, drain_steps=args.drain_steps, reuse_parent_slot=bool(reuse),
                 fuse_interactions=bool(fuse), fuse_along=bool(args.fuse_along),
                 phase_sort=tuple(args.phase_sort) if args.phase_sort else None)
    return s


def time_batch(s, primaries, events):
    import torch
    s.push(primaries)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c = s.run(max_iterations=10_000_000)
    torch.cuda.synchronize()
    return c, time.perf_counter() - t0


def run_variant(w, args, precision, policy, init_partition, prof_kernel, tune=None, drain=None, reuse=None, fuse=None,
                n_initializers=None):
    s = new_session(w, args, precision, policy, init_partition, drain=drain, reuse=reuse, fuse=fuse,
                    n_initializers=n_initializers)
    try:
        events = np.unique(w.primaries["event"])
        tuned = None
        if tune is not None:
            tuned = tune(s)
        for _ in range(args.warmup):
            time_batch(s, w.primaries, events)
            s.release(events)
        c0 = s.counters()
        total_t = 0.0
        iters = 0
        for k in range(args.steps):
            c_before = s.counters()
            c, dt = time_batch(s, w.primaries, events)
            total_t += dt
            iters += c["iterations"] - c_before["iterations"]
            if k + 1 < args.steps or prof_kernel:
                s.release(events)
        c1 = s.counters()
        prof = {}
        work_prof = {}
        if prof_kernel:
            # one more pass over the same batch with HIP events around the kernel
            from paper_2503_17608_amd import emstep
            s.profile(emstep.role_mask(prof_kernel))
            s.profile_read()
            cp0 = s.counters()
            time_batch(s, w.primaries, events)
            cp1 = s.counters()
            prof = s.profile_read()
            s.profile(0)
            work_prof = {k: cp1["work"][k] - cp0["work"][k] for k in cp1["work"]}
        edep, led = s.tallies_by_event(events)
    finally:
        s.close()
    steps = c1["steps"] - c0["steps"]
    work = {k: c1["work"][k] - c0["work"][k] for k in c1["work"]}
    return {"steps": steps, "seconds": total_t, "iterations": iters, "work": work, "prof": prof,
            "work_prof": work_prof, "edep": edep, "ledger": led, "tuned": tuned}


def cpu_baseline(w, n_events):
    import oracle
    import workloads
    sub = workloads.Workload(w.name, w.stack, w.ecut, w.seed, n_events,
                             w.primaries[w.primaries["event"] < n_events], w.n_slots)
    pb = oracle.problem_for(sub)
    tr, rows = oracle.tracks_from_primaries(sub.primaries)
    threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    _, _, steps = pb.run_events(tr, rows, n_events, threads)
    dt = time.perf_counter() - t0
    # one thread on a smaller sample: the per-core rate
    n1 = max(1, min(n_events, n_events // 20))
    sel = sub.primaries["event"] < n1
    t1 = time.perf_counter()
    _, _, steps1 = pb.run_events(tr[sel], rows[sel], n1, 1)
    dt1 = time.perf_counter() - t1
    return {"value": steps / dt, "unit": "track-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_events} events of the workload ({steps} track-steps, {dt:.2f} s wall)",
            "single_core": {"value": steps1 / dt1, "unit": "track-steps/s",
                            "sample": f"first {n1} events ({steps1} track-steps, {dt1:.2f} s)"}}


def fused_along(args, w):
    """Whether the photon and field along-steps run as one launch."""
    return bool(args.fuse_along) and args.streams == 1 and any(b != 0.0 for b in w.stack.B)


def drain_for(args, n_slots):
    """The drain threshold for a session of n_slots slots: the configured one
    at 2^20 slots and above, scaled with the slots below (a fixed threshold
    would drain a small session from its start)."""
    if args.drain_threshold <= 0:
        return 0
    return max(256, min(args.drain_threshold, args.drain_threshold * n_slots // (1 << 20)))


def event_parallel_rate(w, args, precision, k, repeats=2, details=False):
    """Event-parallel mode: k sessions of n_slots/k slots, each on its own
    stream and host thread, events handed out in chunks; track-steps/s."""
    import torch

    from paper_2503_17608_amd import emstep, multistream
    st = w.stack
    # the paper's event-parallel runs hand 16 large events to the streams;
    # here the workload's events are grouped into 16 chunks of equal count
    chunk = max(1, (w.n_events + 15) // 16)
    sessions = []
    for _ in range(k):
        s = emstep.Session(max(w.n_slots // k, 1024), precision=precision, max_events=chunk, max_slabs=st.n_slabs,
                           n_initializers=max(getattr(args, "initializers", 0) // k, 16 * (w.n_slots // k), 1 << 23),
                           max_materials=len(st.materials), seed=w.seed, sort_policy=args.policy,
                           max_substeps=args.max_substeps, graph_iterations=args.graph, lds_tables=args.lds_tables,
                           streams=1, stream=torch.cuda.Stream(), n_primaries=max(len(w.primaries), 1 << 16))
        s.load(st.z_planes, st.slab_material, st.half_width, st.B, st.materials, w.ecut)
        # the same tuning as the mixed-event run, the drain threshold scaled
        # to the session's slots
        s.set_tuning(drain_threshold=drain_for(args, w.n_slots // k), drain_steps=args.drain_steps,
                     fuse_interactions=bool(args.fuse_interactions), fuse_along=bool(args.fuse_along))
        sessions.append(s)
    best = None
    log = []
    try:
        multistream.run_event_parallel(sessions, w.primaries, chunk, keep_results=False)     # warm-up
        for _ in range(repeats):
            torch.cuda.synchronize()
            log = []
            _, _, steps, wall = multistream.run_event_parallel(sessions, w.primaries, chunk, keep_results=False,
                                                               chunk_log=log)
            best = steps / wall if best is None else max(best, steps / wall)
    finally:
        for s in sessions:
            s.close()
    if details:
        n = max(len(log), 1)
        return best, {"sessions": k, "chunk_events": chunk, "chunks": len(log),
                      "iterations_per_chunk": sum(x["iterations"] for x in log) / n,
                      "run_ms_per_chunk": 1e3 * sum(x["run_s"] for x in log) / n,
                      "push_release_ms_per_chunk": 1e3 * sum(x["push_s"] + x["release_s"] for x in log) / n,
                      "chunks_per_session": [sum(1 for x in log if x["session"] == j) for j in range(k)],
                      "wall_s": max((x["end"] for x in log), default=0.0)}
    return best


def measured_copy_gbs(mib=1024, repeats=10):
    """Device-to-device copy bandwidth on this GPU (bytes read + written per
    second), the practical counterpart of the HBM peak."""
    import torch
    src = torch.ones(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(repeats):
        dst.copy_(src)
    t1.record()
    t1.synchronize()
    sec = t0.elapsed_time(t1) / 1e3
    del src, dst
    return 2.0 * repeats * (mib << 20) / sec / 1e9


def path_roofline(work, steps, rate, precision, n_primaries):
    """Whole-path HBM roofline: algorithmic bytes per track-step (every step
    kernel's units of work times its bytes per unit, summed over the batch,
    divided by the steps) times track-steps/s, against the HBM peak.
    Secondaries add their initializer record (the interaction writes it);
    their initialization is counted by the fill."""
    total = sum(kernel_bytes(k, work, precision) for k in ("along_field", "along_neutral", "along_charged",
                                                           "interactions", "init", "drain"))
    secondaries = max(work.get("init", 0) + work.get("reused_slots", 0) - n_primaries, 0)
    total += secondaries * UNIT_BYTES[precision]["secondary"]
    b_step = total / max(steps, 1)
    achieved = rate * b_step / 1e9
    return {"bound": "hbm", "bytes_per_step": b_step, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS}


def layer_error(w, edep):
    """Per-layer mean deposit of `edep` against the FP64 oracle on the same events."""
    import oracle
    pb = oracle.problem_for(w)
    tr, rows = oracle.tracks_from_primaries(w.primaries)
    e_ref, _, _ = pb.run_events(tr, rows, w.n_events, len(os.sched_getaffinity(0)))
    lg = edep.reshape(len(edep), -1, 2).sum(2).mean(0)
    lr = e_ref.reshape(len(e_ref), -1, 2).sum(2).mean(0)
    big = lr >= 0.01 * lr.sum()
    err = np.abs(lg - lr) / np.where(lr > 0, lr, 1.0)
    return {"max_rel_err_layers_ge_1pct": float(err[big].max()), "layers_checked": int(big.sum()),
            "total_rel_err": float(abs(lg.sum() - lr.sum()) / lr.sum())}


def layer_error_events(w, edep, events):
    """Per-layer mean deposit of `edep` (rows = `events`) against the FP64
    oracle on the same events (layers holding >= 1 % of the total)."""
    import oracle
    import workloads
    events = np.asarray(events, dtype=np.int64)
    sel = np.isin(w.primaries["event"].astype(np.int64), events)
    prims = w.primaries[sel].copy()
    remap = {int(e): i for i, e in enumerate(events)}
    # the oracle's rows are 0..n-1; a primary keeps its event id for the
    # random-number key and goes to the row of its position in `events`
    sub = workloads.Workload(w.name, w.stack, w.ecut, w.seed, len(events), prims, w.n_slots)
    pb = oracle.problem_for(sub)
    tr, _ = oracle.tracks_from_primaries(prims)
    rows = np.array([remap[int(e)] for e in prims["event"]], dtype=np.uint32)
    e_ref, _, _ = pb.run_events(tr, rows, len(events), len(os.sched_getaffinity(0)))
    lg = edep.reshape(len(edep), -1, 2).sum(2).mean(0)
    lr = e_ref.reshape(len(e_ref), -1, 2).sum(2).mean(0)
    big = lr >= 0.01 * lr.sum()
    err = np.abs(lg - lr) / np.where(lr > 0, lr, 1.0)
    return {"max_rel_err_layers_ge_1pct": float(err[big].max()), "layers_checked": int(big.sum()),
            "total_rel_err": float(abs(lg.sum() - lr.sum()) / lr.sum())}


def serving_section(args, loads):
    """Continuous batching of the serving workload in mixed precision and in
    FP64: p50/p99 event latency and track-steps/s at arrival rates `loads` x
    the sustained event rate of the closed FP64 batch of the same events
    (all pushed at once, device-resident timing), and the mixed-precision
    serving run's per-layer deposit against the FP64 oracle on a subsample
    of its events."""
    import torch

    import workloads
    from paper_2503_17608_amd import serving
    w = workloads.serving_events(args.serve_events)
    if args.slots:
        w.n_slots = args.slots
    events = serving.split_events(w.primaries)
    ev_ids = np.array([e for e, _ in events], dtype=np.uint64)
    # closed FP64 batch of every event (warmed up on the first 64 events)
    s64 = new_session(w, args, "f64", args.policy, args.init_partition)
    warm = np.concatenate([p for _, p in events[:64]])
    time_batch(s64, warm, None)
    s64.release(ev_ids[:64])
    c_before = s64.counters()["steps"]
    c64, dt64 = time_batch(s64, w.primaries, None)
    s64.release(ev_ids)
    steps64 = c64["steps"] - c_before
    event_rate = len(events) / dt64

    sample = ev_ids[:: max(1, args.serve_sample_every)]

    def one(sess, load, keep):
        arrivals = workloads.poisson_arrival_times(w.seed, load * event_rate, len(events))
        torch.cuda.synchronize()
        res = serving.serve(sess, events, arrivals, track_budget=w.n_slots, iterations_per_poll=max(args.graph, 1),
                            keep_results=keep)
        r = {"load": load, "arrival_rate_hz": load * event_rate,
             "value": res.steps / res.wall_s, "unit": "track-steps/s",
             "latency_ms": {"p50": 1e3 * res.percentile(50), "p99": 1e3 * res.percentile(99),
                            "max": 1e3 * max(res.latency_s.values())},
             "serve_wall_s": res.wall_s, "max_events_in_flight": res.max_in_flight,
             "iterations": res.iterations, "ms_per_iteration": 1e3 * res.wall_s / max(res.iterations, 1)}
        return r, res

    runs = {"mixed": [], "f64": []}
    kept = None
    smx = new_session(w, args, "mixed", args.policy, args.init_partition)
    for k, load in enumerate(loads):
        r, res = one(smx, load, keep=(k == 0))
        if k == 0:
            kept = res
        runs["mixed"].append(r)
    smx.close()
    for load in loads:
        runs["f64"].append(one(s64, load, keep=False)[0])
    s64.close()
    out = {"workload": w.name, "events": len(events), "primaries": int(len(w.primaries)), "n_slots": w.n_slots,
           "closed_fp64_batch": {"value": steps64 / dt64, "unit": "track-steps/s", "seconds": dt64,
                                 "track_steps": steps64, "event_rate_hz": event_rate},
           "arrival_rate": "load x closed_fp64_batch.event_rate_hz (Poisson)", "runs": runs}
    if args.serve_sample_every > 0:
        edep = np.stack([kept.edep[int(e)] for e in sample])
        le = layer_error_events(w, edep, sample)
        le["sample"] = (f"every {args.serve_sample_every}th event of the mixed-precision serving run at load "
                        f"{loads[0]} ({len(sample)} events)")
        out["layer_error_mixed_serving_vs_fp64_oracle"] = le
    return out


def serve_mode(args):
    loads = [args.load] + list(args.extra_loads)
    sv = serving_section(args, loads)
    main_run = sv["runs"]["mixed"][0]
    out = {
        "metric": "event latency p50/p99 and track-steps/s, continuous batching",
        "value": main_run["value"], "unit": "track-steps/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": sv["workload"], "events": sv["events"], "primaries": sv["primaries"],
                   "n_slots": sv["n_slots"], "load": args.load, "sort_policy": args.policy,
                   "graph_iterations": args.graph},
        "latency_ms": main_run["latency_ms"],
        "serving": sv,
    }
    print(json.dumps(out), flush=True)


def io_inclusive_rate(w, args, precision):
    """The main configuration timed from the push of the primaries (host
    buffer -> device) to the readback of every event's tallies (device ->
    host): the PCIe-inclusive rate, beside the device-resident `value`."""
    import torch
    s = new_session(w, args, precision, args.policy, args.init_partition)
    events = np.unique(w.primaries["event"])
    time_batch(s, w.primaries, events)
    s.release(events)
    tot, steps = 0.0, 0
    for _ in range(args.steps):
        c0 = s.counters()["steps"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.push(w.primaries)
        c = s.run(max_iterations=10_000_000)
        s.tallies_by_event(events)
        tot += time.perf_counter() - t0
        steps += c["steps"] - c0
        s.release(events)
    s.close()
    return {"value": steps / tot, "unit": "track-steps/s", "ms_per_step": 1e3 * tot / args.steps,
            "timed": "push of the primaries + stepping until empty + readback of every event's tallies"}


def extras(args, w, precision, value, out):
    """The rest of the metric in the same run: unsorted stepping with every
    other setting equal, the PCIe-inclusive rate, mixed precision against
    FP64 on the mixed-species cone workload (with its per-layer error
    against the FP64 oracle), and the serving loop in both precisions."""
    import workloads
    t0 = time.perf_counter()
    rv = run_variant(w, args, precision, "none", args.init_partition, None)
    unsorted = rv["steps"] / rv["seconds"]
    out["unsorted"] = {"sort_policy": "none", "value": unsorted, "unit": "track-steps/s",
                       "sorted_over_unsorted": value / unsorted,
                       "same_as_main": "every setting except the sort policy",
                       "track_steps_per_step": rv["steps"] // args.steps}
    out["io_inclusive"] = io_inclusive_rate(w, args, precision)
    wc = workloads.mixed_cone_showers()
    pair = {"workload": wc.name, "events": wc.n_events, "n_slots": wc.n_slots}
    for prec in ("f64", "mixed"):
        rc = run_variant(wc, args, prec, args.policy, args.init_partition, None)
        pair[prec] = {"value": rc["steps"] / rc["seconds"], "unit": "track-steps/s",
                      "track_steps_per_step": rc["steps"] // args.steps}
        if prec == "mixed":
            pair["layer_error_mixed_vs_fp64_oracle"] = layer_error(wc, rc["edep"])
    pair["mixed_over_f64"] = pair["mixed"]["value"] / pair["f64"]["value"]
    out["precision_pair"] = pair
    out["serving"] = serving_section(args, [0.5, 0.7, 0.9])
    out["extras_wall_s"] = time.perf_counter() - t0


def fig2_mode(args):
    """Along-step GPU time per live track against the number of live tracks
    (one iteration at a time, per-kernel HIP events, no drain), the tail
    onset, and the whole batch timed with and without the drain of the last
    tracks (graphs on, device-resident timing)."""
    from paper_2503_17608_amd import trace
    w = make_workload(args.workload, args.events, args.slots)
    precision = args.precision or w.precision
    s = new_session(w, args, precision, args.policy, args.init_partition, graph=0, drain=0)
    recs = trace.record(s, w.primaries)
    s.close()
    if args.trace_out:
        trace.write(recs, args.trace_out, name=f"{w.name} {args.policy}")
    an = trace.tail_analysis(recs)
    thr = args.drain_threshold if args.drain_threshold > 0 else 65536
    tail = [r for r in recs if r["alive"] + r["queued"] + r["pending"] < thr]
    tail_ms = sum(sum(r["kernel_ms"].values()) for r in tail)
    rd = run_variant(w, args, precision, args.policy, args.init_partition, None, drain=thr)
    rn = run_variant(w, args, precision, args.policy, args.init_partition, None, drain=0)
    out = {"metric": "along-step time per live track against live tracks", "n_gpus": 1,
           "config": {"workload": w.name, "events": w.n_events, "n_slots": w.n_slots, "precision": precision,
                      "sort_policy": args.policy, "init_partition": args.init_partition},
           "iterations": len(recs), "track_steps": sum(r["steps"] for r in recs),
           "tail_analysis": an,
           "below_drain_threshold": {"threshold": thr, "iterations": len(tail), "kernel_ms": tail_ms,
                                     "share_of_kernel_time": tail_ms / an["kernel_ms"]},
           "batch_with_drain": {"value": rd["steps"] / rd["seconds"], "ms_per_batch": 1e3 * rd["seconds"] / args.steps,
                                "iterations_per_batch": rd["iterations"] // args.steps},
           "batch_without_drain": {"value": rn["steps"] / rn["seconds"],
                                   "ms_per_batch": 1e3 * rn["seconds"] / args.steps,
                                   "iterations_per_batch": rn["iterations"] // args.steps}}
    print(json.dumps(out), flush=True)


def sweep_mode(args):
    """Throughput against the total number of track slots: the mixed-event
    mode (every event in one slot array on one stream) and the event-parallel
    mode (k sessions of slots / k, each on its own stream and host thread,
    events from a shared queue), k = 2, 4, 8."""
    w = make_workload(args.workload, args.events, args.slots)
    precision = args.precision or w.precision
    rows = []
    lo, hi = args.sweep_exp
    for e in range(lo, hi + 1):
        n = 1 << e
        w.n_slots = n
        t0 = time.perf_counter()
        # few slots hold back many secondaries: the initializer buffer is
        # sized for the whole workload's peak, not for the slots
        from paper_2503_17608_amd.emstep import EmsError
        row = {"slots": n}
        try:
            r = run_variant(w, args, precision, args.policy, args.init_partition, None, drain=drain_for(args, n),
                            n_initializers=args.initializers or max(16 * n, 1 << 24))
            row.update({"mixed": r["steps"] / r["seconds"], "mixed_iterations_per_batch": r["iterations"] // args.steps})
        except EmsError as e:          # e.g. more secondaries waiting than the initializer buffer holds
            row["mixed_error"] = str(e)
        for k in args.sweep_k:
            if n // k >= 1024:
                try:
                    row[f"event_parallel_{k}"], row[f"event_parallel_{k}_detail"] = event_parallel_rate(
                        w, args, precision, k, repeats=1, details=True)
                except EmsError as e:
                    row[f"event_parallel_{k}_error"] = str(e)
        row["wall_s"] = time.perf_counter() - t0
        print(json.dumps(row), flush=True)
        rows.append(row)
    out = {"metric": "track-steps/s against total track slots", "unit": "track-steps/s", "n_gpus": 1,
           "config": {"workload": w.name, "events": w.n_events, "precision": precision, "sort_policy": args.policy},
           "rows": rows}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the transport shards by event "
              "and no multi-GPU figure is produced.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    if args.calibrate_copy_mib > 0:
        src = torch.ones(args.calibrate_copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.serve:
        serve_mode(args)
        return
    if args.fig2:
        fig2_mode(args)
        return
    if args.sweep:
        sweep_mode(args)
        return
    w = make_workload(args.workload, args.events, args.slots)
    precision = args.precision or w.precision
    prof_kernel = None if args.no_roofline else args.roofline_kernel
    tune = None
    if args.autotune:
        from paper_2503_17608_amd import autotune
        # tuned on the whole workload: a fraction of the events would not fill
        # the slots as the full run does, and at low occupancy the masked
        # policy and no drain look best (1/8 of the default workload chose
        # them, 1.38e9 against 2.54e9 track-steps/s for the defaults)
        tune = lambda s: autotune.autotune(s, w.primaries)  # noqa: E731
    r = run_variant(w, args, precision, args.policy, args.init_partition, prof_kernel, tune)
    value = r["steps"] / r["seconds"]
    out = {
        "metric": "track-steps/s",
        "value": value,
        "unit": "track-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r["seconds"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "f64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "events": w.n_events, "primaries": int(len(w.primaries)),
                   "n_slots": w.n_slots, "sort_policy": args.policy, "init_partition": args.init_partition,
                   "max_substeps": args.max_substeps, "graph_iterations": args.graph,
                   "lds_tables": args.lds_tables, "streams": args.streams,
                   "drain_threshold": args.drain_threshold, "drain_steps": args.drain_steps,
                   "reuse_parent_slot": args.reuse_parent_slot, "fuse_interactions": args.fuse_interactions,
                   "fuse_along": int(fused_along(args, w)),
                   "phase_sort": ["0x%08X" % m for m in args.phase_sort],
                   "track_steps_per_step": r["steps"] // args.steps,
                   "iterations_per_step": r["iterations"] // args.steps},
        "work_per_step": {k: v // args.steps for k, v in r["work"].items()},
    }
    if r["tuned"] is not None:
        out["config"]["autotuned"] = {k: r["tuned"][k] for k in ("sort_policy", "tail_threshold", "block",
                                                                 "fuse_interactions", "fuse_along", "drain_threshold",
                                                                 "phase_sort")}
        out["config"]["autotuned"]["phase_choice"] = r["tuned"].get("phase_table", {}).get("choice")
    if prof_kernel and r["prof"].get(prof_kernel, (0, 0))[1] > 0:
        ms, launches = r["prof"][prof_kernel]
        # with fuse_along the field role's launch (k_along_both) also steps
        # the photons: its bytes and tracks are both along-steps'
        both = prof_kernel == "along_field" and fused_along(args, w)
        parts = ("along_field", "along_neutral") if both else (prof_kernel,)
        tracks = sum(r["work_prof"][k] for k in parts)
        avg_s = ms / 1e3 / launches
        per_launch = sum(kernel_bytes(k, r["work_prof"], precision) for k in parts) / launches
        bpt = per_launch * launches / max(tracks, 1)
        achieved = per_launch / avg_s / 1e9
        key = {"workload": w.name, "precision": precision, "n_slots": w.n_slots, "sort_policy": args.policy,
               "init_partition": args.init_partition, "max_substeps": args.max_substeps,
               "drain_threshold": args.drain_threshold, "reuse_parent_slot": args.reuse_parent_slot,
               "fuse_interactions": args.fuse_interactions, "fuse_along": int(both),
               "phase_sort": ["0x%08X" % m for m in args.phase_sort]}
        label = "along_both" if both else prof_kernel
        t = committed_traffic(label, key)
        out["roofline"] = {"bound": "hbm", "kernel": label, "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": t["bytes_per_launch"] if t else None,
                           "traffic_unit": "bytes/launch (calibrated FETCH_SIZE + WRITE_SIZE)",
                           "algorithmic_bytes_per_launch": per_launch,
                           "avg_launch_us": avg_s * 1e6, "launches": launches,
                           "tracks_per_launch": tracks / launches, "bytes_per_track": bpt,
                           "timing": "HIP start/stop events stamped by the kernel's own dispatch packet "
                                     "(hipExtLaunchKernel) on every launch of the kernel, in one extra pass over "
                                     "the same batch (graph replay off for that pass)"}
    out["path_roofline"] = path_roofline(r["work"], r["steps"], value, precision, args.steps * len(w.primaries))
    if not args.no_roofline and args.calibrate_copy_mib == 0:
        # (counter runs leave it out: their only copies are the calibration's)
        copy_gbs = measured_copy_gbs()
        out["path_roofline"]["measured_copy_gbs"] = copy_gbs
        out["path_roofline"]["frac_of_measured_copy"] = out["path_roofline"]["achieved"] / copy_gbs
        if "roofline" in out:
            out["roofline"]["measured_copy_gbs"] = copy_gbs
            out["roofline"]["frac_of_measured_copy"] = out["roofline"]["achieved"] / copy_gbs
    if args.compare:
        var = {}
        for pol, part, dr, ru in [("none", 0, None, None), ("none", 1, None, None), ("partition", 0, None, None),
                                  ("partition", 1, None, None), ("radix", 0, None, None), ("queue", 0, None, None),
                                  ("none", 0, 0, None), ("partition", 1, 0, None), ("partition", 0, None, 1),
                                  ("partition", 1, None, 1)]:
            if pol == args.policy and part == args.init_partition and dr is None and ru is None:
                continue
            rv = run_variant(w, args, precision, pol, part, None, drain=dr, reuse=ru)
            tag = f"{pol}+part{part}" + ("+nodrain" if dr == 0 else "") + ("+reuse" if ru else "")
            var[tag] = rv["steps"] / rv["seconds"]
        for pol in ("partition", "radix", "none"):
            fu = 0 if args.fuse_interactions else 1
            part = args.init_partition if pol == args.policy else 0
            rv = run_variant(w, args, precision, pol, part, None, fuse=fu)
            tag = f"{pol}+part{part}" + ("+fused" if fu else "+unfused")
            var[tag] = rv["steps"] / rv["seconds"]
        for k in (2, 4, 8, 16):
            var[f"event_parallel_{k}x{w.n_slots // k}"] = event_parallel_rate(w, args, precision, k)
        out["variants"] = var
    if args.layer_error:
        out["layer_error_vs_fp64_oracle"] = layer_error(w, r["edep"])
    if not args.no_extras and not args.autotune and args.workload == "electron_showers_1gev_field":
        extras(args, w, precision, value, out)
    if args.cpu_events > 0:
        out["cpu_baseline"] = cpu_baseline(w, min(args.cpu_events, w.n_events))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
