"""Benchmark of the kernel-style N-turn planner hot path on one MI355X.

One step = one whole plan of the 512 x 512 x 512 maze with N = 20 maneuver
cycles, inputs resident in HBM: obstacle rendering, init, 120 maneuver
sweeps, goal search and back-tracking (the planner object and its tables are
made once, before timing, like the paper's `ini`).

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  `value` is pose-cell updates per second over whole
steps (6 N N_R updates per plan); plans/s, sweep-only throughput, per-stage
times and p50/p99 plan latency ride along.  The sweeps run as the passes
sweep_n_turns groups them into (two turns on shared circles fused into one
pass), one event per pass; `roofline` covers the pass kind with the largest
share of the step, from HIP events recorded on the plan's stream during the
timed steps; `cpu_baseline` times the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pose-cell updates/s and plans/s at 512³ N=20; p50/p99 plan latency batched vs single"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = 9  # read V (4 B) + read obstacle code (1 B) + write V (4 B), per pose and pass
TURNS = (0, 2, 3, 5)   # LF, RB, RF, LB
# pass kinds: the kernels one pass of each kind launches
PASS_KINDS = {
    "fused_turn": "row_sweep_kernel<32, true, false, true> (two turn maneuvers on shared circles in one pass)",
    "turn": "row_sweep_kernel<32, false, false, true> (one turn maneuver)",
    "straight": "row_sweep_kernel<32, false, false, true> (y-major planes) + xmajor_sweep_kernel<32, 256> (x-major planes)",
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sweeps_maze_512.json")


def pass_kind(first: int, second: int) -> str:
    if second >= 0:
        return "fused_turn"
    return "turn" if first in TURNS else "straight"



def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("k_sweep.hip", "nhp_internal.h"):
        with open(os.path.join(ROOT, "paper_2306_01301_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kind: str):
    """HBM bytes per pass of this kind from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_pass", {}).get(kind)


def cpu_model() -> str:
    try:
        out = subprocess.check_output(["lscpu"], text=True)
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(scene, cycles: int):
    """The oracle as it stands, on the host's cores, on `cycles` maneuver
    cycles of the same workload (a bounded sample of the 20)."""
    import oracle

    oracle.build()
    threads = oracle.set_threads(os.cpu_count() or 1)
    prob = oracle.Problem(scene.nx, scene.nt, scene.R, scene.half_cell, list(scene.schedule), list(scene.ct),
                          list(scene.gear))
    B = oracle.render(prob, scene.image, *scene.vehicle)
    V = oracle.init(prob, B, scene.start)
    t0 = time.perf_counter()
    oracle.cycles(prob, B, V, cycles)
    dt = time.perf_counter() - t0
    updates = len(scene.schedule) * cycles * scene.n_poses
    return {"value": updates / dt, "unit": "pose-cell updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d of %d maneuver cycles (%d sweeps, %.2e pose updates) of %s on %d threads of %s, %.1f s"
                      % (cycles, scene.n_cycles, len(scene.schedule) * cycles, updates, scene.name, threads,
                         cpu_model(), dt)}


def batch_comparison() -> dict:
    """64 mixed planning instances submitted at once: one plan per launch vs
    shared launches.  Latency of a plan = completion - submission."""
    from paper_2306_01301_amd import scenes, serving, sizing

    reqs = scenes.batch_64()
    updates = sum(sizing.pose_updates(s.nx, s.nt, s.n_cycles, len(s.schedule)) for s in reqs)
    serving.run_batched(reqs[:8])  # warm-up
    serving.run_single(reqs[:8])
    out = {"workload": "batch_64", "plans": len(reqs), "pose_updates": updates}

    def continuous(rs):
        srv = serving.Server(1 << 60, max_live=len(rs))
        res = srv.run(rs, [0.0] * len(rs))
        srv.close()
        return res

    # three runs of each mode, interleaved; the run with the median throughput is reported
    runs = {"one_plan_per_launch": [], "batched": [], "continuous": []}
    for _ in range(3):
        for name, fn in (("one_plan_per_launch", serving.run_single), ("batched", serving.run_batched),
                         ("continuous", continuous)):
            res = fn(reqs)
            s = serving.latency_summary(res)
            s["pose_updates_per_s"] = updates / max(r.finished for r in res)
            runs[name].append(s)
    for name, ss in runs.items():
        ss.sort(key=lambda s: s["plans_per_s"])
        out[name] = dict(ss[len(ss) // 2], runs=len(ss))
    return out


def bench_serving(args) -> int:
    """Continuous batching under Poisson arrivals of mixed requests (sides up
    to 1024, headings up to 512, N up to 20), admitted by HBM footprint."""
    import torch

    from paper_2306_01301_amd import scenes, serving, sizing

    reqs = scenes.serving_requests(count=args.requests)
    free, total = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    rates = [float(r) for r in args.rates.split(",") if r]
    warm = serving.Server(budget, max_live=64)
    warm.run(reqs[:4], [0.0] * 4)
    warm.close()
    per_rate = []
    for rate in rates:
        arr = scenes.poisson_arrivals(1306 + int(rate), rate, len(reqs))
        srv = serving.Server(budget, max_live=64)
        res = srv.run(reqs, arr)
        srv.close()
        s = serving.latency_summary(res)
        s["rate"] = rate
        s["one_plan_at_a_time"] = serving.latency_summary(serving.run_fifo(reqs, arr))
        per_rate.append(s)
        print(json.dumps({"rate": rate, **{k: v for k, v in s.items() if k != "rate"}}), file=sys.stderr, flush=True)
    updates = sum(sizing.pose_updates(s.nx, s.nt, s.n_cycles, len(s.schedule)) for s in reqs)
    best = max(per_rate, key=lambda s: s["plans_per_s"] or 0)
    out = {"metric": METRIC, "value": best["plans_per_s"], "unit": "plans/s", "n_gpus": 1, "steps": len(rates),
           "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u32", "data": "synthetic",
           "config": {"workload": "serving_requests", "requests": len(reqs), "pose_updates": updates,
                      "hbm_budget_bytes": budget, "admission": "25 B/pose (3 vertices x 2 gears x 4 B + 1 B)"},
           "serving": per_rate}
    print(json.dumps(out), flush=True)
    return 0


def bench_reach(args) -> int:
    """Maneuver-count reachability (App. C) on the 128 x 128 x 512, N = 8
    workload: one step renders the obstacle bits, runs the cycles and
    extracts the plan."""
    import torch

    from paper_2306_01301_amd import planner, scenes, sizing

    sc = scenes.WORKLOADS[args.workload]()
    p = planner.planner_for(sc)
    rc = planner.Reach(p, sc.n_cycles)
    image = torch.from_numpy(np.ascontiguousarray(sc.image)).cuda()
    stream = p.stream

    def one(events):
        def mark(tag):
            if events is not None:
                e = torch.cuda.Event(enable_timing=True)
                e.record(stream)
                events.append((tag, e))
        mark("start")
        rc.render(image, sc.vehicle)
        mark("render")
        rc.sweep(sc.start, sc.n_cycles)
        mark("sweep")
        path = rc.extract(sc.goal, sc.goal_radius)
        mark("extract")
        return path

    for _ in range(args.warmup):
        one(None)
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev = []
        path = one(ev)
        evs.append(ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = {}
    for ev in evs:
        for (a, ea), (b, eb) in zip(ev[:-1], ev[1:]):
            stages.setdefault(b, []).append(ea.elapsed_time(eb))
    ms = 1000.0 * wall / args.steps
    updates = sizing.pose_updates(sc.nx, sc.nt, sc.n_cycles, len(sc.schedule))
    out = {"metric": "maneuver-count reachability plans/s at 128x128x512 N=8 (App. C)", "value": 1000.0 / ms,
           "unit": "plans/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32 bit-vectors",
           "data": "synthetic",
           "config": {"workload": sc.name, "grid": [sc.nx, sc.nx, sc.nt], "n_cycles": sc.n_cycles,
                      "pose_updates_per_plan": updates},
           "pose_updates_per_s": updates / (ms * 1e-3),
           "stages_ms": {k: float(np.median(v)) for k, v in stages.items()},
           "plan": {"maneuvers": path.level, "best": list(path.best)},
           "paper_context": "Table 9: about 2 ms per 8-cycle plan at 128x128x512 on the paper's larger GPU"}
    if args.cpu_cycles > 0:
        import oracle

        oracle.build()
        threads = oracle.set_threads(os.cpu_count() or 1)
        prob = oracle.Problem(sc.nx, sc.nt, sc.R, sc.half_cell, list(sc.schedule), list(sc.ct), list(sc.gear))
        B = oracle.render(prob, sc.image, *sc.vehicle)
        t1 = time.perf_counter()
        oracle.reach(prob, B, sc.start, sc.n_cycles)
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": 1.0 / dt, "unit": "plans/s", "cores": threads, "kind": "oracle",
                               "sample": "the reachability cycles of one %s plan (%d cycles) on %d threads of %s, "
                                         "%.2f s" % (sc.name, sc.n_cycles, threads, cpu_model(), dt)}
    rc.close()
    p.close()
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="maze_512")
    ap.add_argument("--cpu-cycles", type=int, default=20, help="oracle cycles timed for cpu_baseline (0: skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain device copy of 1 GiB (counter calibration)")
    ap.add_argument("--skip-batch", action="store_true", help="skip the batched-vs-single comparison")
    ap.add_argument("--rates", default="10,20,50,100,200,500",
                    help="serving workload: Poisson arrival rates in plans/s")
    ap.add_argument("--requests", type=int, default=48, help="serving workload: requests per rate")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        return 2

    import torch

    from paper_2306_01301_amd import planner, scenes, sizing

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload.startswith("reach"):
        return bench_reach(args)
    sc = scenes.WORKLOADS[args.workload]()
    if args.calibrate_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    p = planner.planner_for(sc)
    image = torch.from_numpy(np.ascontiguousarray(sc.image)).cuda()
    stream = p.stream
    n_sched = len(sc.schedule)
    passes = planner.schedule_passes(sc.schedule, 0, n_sched * sc.n_cycles)

    def one_plan(events):
        """One step.  events: list to append (tag, event) pairs to, or None."""
        def mark(tag):
            if events is not None:
                e = torch.cuda.Event(enable_timing=True)
                e.record(stream)
                events.append((tag, e))
        mark("start")
        p.render(image, sc.vehicle)
        mark("render")
        p.sweep(sc.start, 0)  # init: V = INF, V(start) = 0
        mark("init")
        for a, b in passes:  # the passes sweep_n_turns runs, one event each
            p.sweep_pass(a, b)
            mark((a, b))
        path = p.extract(sc.goal, sc.goal_radius, sc.w_xy, sc.w_t)
        mark("extract")
        return path

    for _ in range(args.warmup):
        one_plan(None)
    torch.cuda.synchronize()

    step_events = []
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev = []
        ts = time.perf_counter()
        path = one_plan(ev)
        lat.append(time.perf_counter() - ts)  # extract synchronises: submission to plan on the host
        step_events.append(ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # per-stage and per-pass durations from the events (plan's stream)
    stage = {"render": [], "init": [], "sweeps": [], "extract": []}
    kinds = {k: [] for k in PASS_KINDS}
    for ev in step_events:
        t = {}
        prev = None
        sweeps = 0.0
        for tag, e in ev:
            if prev is not None:
                dt = prev[1].elapsed_time(e)
                if tag in ("render", "init", "extract"):
                    t[tag] = dt
                else:
                    sweeps += dt
                    kinds[pass_kind(*tag)].append(dt)
            prev = (tag, e)
        for k in ("render", "init", "extract"):
            stage[k].append(t[k])
        stage["sweeps"].append(sweeps)

    updates = sizing.pose_updates(sc.nx, sc.nt, sc.n_cycles, n_sched)
    ms_per_step = 1000.0 * wall / args.steps
    # every pass reads V and the codes and writes V once per pose
    alg_bytes = BYTES_PER_UPDATE * sc.n_poses
    per_kind = {}
    for k, v in kinds.items():
        if v:
            avg = float(np.mean(v))
            per_kind[k] = {"passes_per_step": len(v) // args.steps, "avg_ms": avg,
                           "ms_per_step": float(np.sum(v)) / args.steps,
                           "GB_per_s": alg_bytes / (avg * 1e-3) / 1e9,
                           "updates_per_pose": 2 if k == "fused_turn" else 1, "kernel": PASS_KINDS[k]}
    # the dominant kernel: a straight pass is two kernels (y-major and x-major
    # planes), each with a smaller share than a pass kind of one kernel
    dom = max((k for k in per_kind if k != "straight"), key=lambda k: per_kind[k]["ms_per_step"])
    achieved = per_kind[dom]["GB_per_s"]
    sweep_ms = float(np.median(stage["sweeps"]))
    lat_ms = np.array(lat) * 1000.0
    out = {
        "metric": METRIC,
        "value": updates / (ms_per_step * 1e-3),
        "unit": "pose-cell updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": sc.name, "grid": [sc.nx, sc.nx, sc.nt], "n_cycles": sc.n_cycles,
                   "sweeps_per_plan": n_sched * sc.n_cycles, "pose_updates_per_plan": updates,
                   "vehicle_box_frs": list(sc.vehicle), "turn_radius_cells": sc.R, "plans_per_step": 1},
        "plans_per_s": 1000.0 / ms_per_step,
        "sweep_updates_per_s": updates / (sweep_ms * 1e-3),
        "latency_ms": {"single": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
                       "batched": None},
        "stages_ms": {k: float(np.median(v)) for k, v in stage.items()},
        "plan": {"maneuvers": len(path.steps), "cost_cells": path.value / 1024.0, "best": list(path.best)},
        "roofline": {"kernel": PASS_KINDS[dom], "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom), "bytes_per_launch_algorithmic": alg_bytes,
                     "avg_launch_ms": per_kind[dom]["avg_ms"], "launches_timed": len(kinds[dom]),
                     "passes": per_kind},
    }
    p.close()
    if not args.skip_batch:
        out["latency_ms"]["batch_64"] = batch_comparison()
    if args.cpu_cycles > 0:
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_cycles)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
