"""Benchmark: track-steps/s of the step-based EM shower loop on one MI355X.

One benchmark step is one pass of the whole hot path over one batch: every
primary of the workload transported until no track is alive, queued or
pending (vacancy compaction, initialization, pre-step, sort, along-step,
interactions, tallies).  Primaries are copied to the device before the timed
region of each step; the timed region covers the device loop only.

Default workload: 10^4 electrons of 1 GeV into a 50-layer Pb (2 mm) / liquid
Ar (5 mm) stack, 40 x 40 cm, uniform 1 T field along x, 0.1 MeV cut, 2^20
track slots, FP64.

The JSON line carries the dominant kernel's roofline (algorithmic bytes per
launch from the kernel's work counters and its per-track field traffic,
divided by its average launch duration measured with HIP events on the
library's stream during the timed steps) and the oracle's throughput on the
host cores for a bounded sample of the same events.
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

# Algorithmic bytes per processed track for each kernel (SoA fields read and
# written for a participating track, plus 16 B of tally read-modify-write for
# charged steps), FP64 / mixed.  Derivation in the design doc.
BYTES_PER_TRACK = {
    "f64": {"pre_step": 62, "along_neutral": 148, "along_charged": 164, "along_field": 222,
            "compton": 122, "photoelectric": 122, "pair": 122, "moller": 122, "bhabha": 122,
            "bremsstrahlung": 122, "init": 206},
    "mixed": {"pre_step": 46, "along_neutral": 124, "along_charged": 140, "along_field": 178,
              "compton": 102, "photoelectric": 102, "pair": 102, "moller": 102, "bhabha": 102,
              "bremsstrahlung": 102, "init": 174},
}

WORKLOADS = {
    "electron_showers_1gev_field": "electron_showers_1gev_field",
    "small_electron_showers": "small_electron_showers",
    "mixed_cone_showers": "mixed_cone_showers",
    "batched_mixed_events": "batched_mixed_events",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="electron_showers_1gev_field", choices=sorted(WORKLOADS))
    ap.add_argument("--events", type=int, default=0, help="override the number of events")
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--precision", default="", choices=["", "f64", "mixed"])
    ap.add_argument("--policy", default="queue", choices=["none", "partition", "radix", "queue"])
    ap.add_argument("--init-partition", type=int, default=0)
    ap.add_argument("--max-substeps", type=int, default=10)
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--graph", type=int, default=0, help="iterations per captured HIP graph (0 = plain launches)")
    ap.add_argument("--lds-tables", type=int, default=1)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--roofline-kernel", default="along_field")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--cpu-events", type=int, default=4000, help="oracle sample (events); 0 = skip")
    ap.add_argument("--compare", action="store_true", help="also time the other sort policies")
    return ap.parse_args()


def make_workload(name, events, slots):
    import workloads
    kw = {}
    if events:
        kw["n_events"] = events
    w = getattr(workloads, WORKLOADS[name])(**kw)
    if slots:
        w.n_slots = slots
    return w


def run_variant(w, args, precision, policy, init_partition, prof_kernel):
    import torch

    from paper_2503_17608_amd import emstep
    st = w.stack
    s = emstep.Session(w.n_slots, precision=precision, max_events=w.n_events, max_slabs=st.n_slabs,
                       max_materials=len(st.materials), seed=w.seed, sort_policy=policy,
                       init_partition=init_partition, max_substeps=args.max_substeps, block_size=args.block_size,
                       graph_iterations=args.graph, lds_tables=args.lds_tables, streams=args.streams,
                       n_primaries=max(len(w.primaries), 1 << 16))
    s.load(st.z_planes, st.slab_material, st.half_width, st.B, st.materials, w.ecut)
    events = np.unique(w.primaries["event"])

    def one_step():
        s.push(w.primaries)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = s.run(max_iterations=10_000_000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return c, dt

    for _ in range(args.warmup):
        one_step()
        for e in events:
            s.release(int(e))
    if prof_kernel:
        s.profile(emstep.role_mask(prof_kernel))
        s.profile_read()          # clear
    c0 = s.counters()
    total_t = 0.0
    iters = 0
    for k in range(args.steps):
        c_before = s.counters()
        c, dt = one_step()
        total_t += dt
        iters += c["iterations"] - c_before["iterations"]
        if k + 1 < args.steps:
            for e in events:
                s.release(int(e))
    c1 = s.counters()
    prof = s.profile_read() if prof_kernel else {}
    # one last correctness look: the energy ledger of the final step
    edep, led = s.tallies_by_event(events)
    s.close()
    steps = c1["steps"] - c0["steps"]
    work = {k: c1["work"][k] - c0["work"][k] for k in c1["work"]}
    return {"steps": steps, "seconds": total_t, "iterations": iters, "work": work, "prof": prof,
            "edep_total": float(edep.sum()), "escaped": float(led["escaped"].sum())}


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
    return {"value": steps / dt, "unit": "track-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_events} events of the workload ({steps} track-steps, {dt:.2f} s wall)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the transport shards by event "
              "and no multi-GPU figure is produced.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    w = make_workload(args.workload, args.events, args.slots)
    precision = args.precision or w.precision
    prof_kernel = None if args.no_roofline else args.roofline_kernel
    r = run_variant(w, args, precision, args.policy, args.init_partition, prof_kernel)
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
                   "track_steps_per_step": r["steps"] // args.steps,
                   "iterations_per_step": r["iterations"] // args.steps},
        "work_per_step": {k: v // args.steps for k, v in r["work"].items()},
    }
    if prof_kernel and r["prof"].get(prof_kernel, (0, 0))[1] > 0:
        ms, launches = r["prof"][prof_kernel]
        tracks = r["work"][prof_kernel]
        bpt = BYTES_PER_TRACK[precision][prof_kernel]
        avg_s = ms / 1e3 / launches
        per_launch = tracks * bpt / launches
        achieved = per_launch / avg_s / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": prof_kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                           "avg_launch_us": avg_s * 1e6, "launches": launches,
                           "tracks_per_launch": tracks / launches, "bytes_per_track": bpt}
    if args.compare:
        var = {}
        for pol, part in [("none", 0), ("none", 1), ("partition", 0), ("partition", 1), ("radix", 0),
                          ("queue", 0), ("queue", 1)]:
            if pol == args.policy and part == args.init_partition:
                continue
            rv = run_variant(w, args, precision, pol, part, None)
            var[f"{pol}+part{part}"] = rv["steps"] / rv["seconds"]
        out["variants"] = var
    if args.cpu_events > 0:
        out["cpu_baseline"] = cpu_baseline(w, min(args.cpu_events, w.n_events))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
