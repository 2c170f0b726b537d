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
# the sweep kernels of the maze workload (512-pose curves: 32-step sections)
KERNELS = {
    "fused_turn": "row_sweep_kernel<32, true, false, true, true> (two turn maneuvers on shared circles in one launch)",
    "turn": "row_sweep_kernel<32, false, false, true, true> (one turn maneuver)",
    "straight_y": "row_sweep_kernel<32, false, false, true, false> (straight maneuver, y-major planes)",
    "straight_x": "xmajor_band_kernel<32, 256, 1> (straight maneuver, x-major planes, band tiles)",
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sweeps_maze_512.json")


def kernel_kind(first: int, second: int) -> str:
    if second >= 0:
        return "fused_turn"
    return "turn" if first in TURNS else "straight"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("k_sweep.hip", "nhp_internal.h"):
        with open(os.path.join(ROOT, "paper_2306_01301_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of each sweep kernel from the committed rocprofv3
    counter summary, or {} when the kernel source changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {}
    if t.get("kernel_source_hash") != kernel_source_hash():
        return {}
    return t.get("bytes_per_launch", {})


def host_cpu() -> dict:
    """The host's processor as lscpu and /proc/cpuinfo name it, and the CPUs
    this process may run on."""
    info = {"nproc": None, "os_cpu_count": os.cpu_count(), "affinity": None, "lscpu_model": None,
            "cpuinfo_model": None, "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        info["nproc"] = int(subprocess.check_output(["nproc"], text=True).strip())
    except Exception:
        pass
    try:
        out = subprocess.check_output(["lscpu"], text=True)
        for line in out.splitlines():
            key, _, val = line.partition(":")
            if key.strip() in ("Model name", "Vendor ID", "CPU family", "Model", "Thread(s) per core",
                               "Core(s) per socket", "Socket(s)", "CPU(s)"):
                info.setdefault("lscpu", {})[key.strip()] = val.strip()
                if key.strip() == "Model name":
                    info["lscpu_model"] = val.strip()
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpuinfo_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return info


def cpu_baseline(scene, cycles_all: int, cycles_one: int):
    """The oracle as it stands, built -O3 -march=native -fopenmp on the host
    it runs on: all 20 cycles on all the host CPUs this process may use, and
    a bounded sample of the cycles on one core."""
    import oracle

    lib = oracle.build(native=True)
    prob = oracle.Problem(scene.nx, scene.nt, scene.R, scene.half_cell, list(scene.schedule), list(scene.ct),
                          list(scene.gear))
    host = host_cpu()
    want = host["affinity"] or os.cpu_count() or 1
    if host["omp_num_threads"]:
        want = min(want, int(host["omp_num_threads"]))
    B = oracle.render(prob, scene.image, *scene.vehicle)
    V0 = oracle.init(prob, B, scene.start)
    runs = {}
    for name, threads, cycles in (("all", want, cycles_all), ("one", 1, cycles_one)):
        if cycles <= 0:
            continue
        used = oracle.set_threads(threads)
        V = V0.copy()
        t0 = time.perf_counter()
        oracle.cycles(prob, B, V, cycles)
        dt = time.perf_counter() - t0
        updates = len(scene.schedule) * cycles * scene.n_poses
        runs[name] = {"value": updates / dt, "unit": "pose-cell updates/s", "cores": used, "seconds": dt,
                      "sample": "%d of %d maneuver cycles (%d sweeps, %.2e pose updates) of %s on %d thread%s"
                                % (cycles, scene.n_cycles, len(scene.schedule) * cycles, updates, scene.name, used,
                                   "" if used == 1 else "s")}
    oracle.set_threads(want)
    main = runs.get("all") or runs.get("one")
    model = host["lscpu_model"] or host["cpuinfo_model"] or platform.processor() or "unknown"
    return {"value": main["value"], "unit": main["unit"], "cores": main["cores"], "kind": "oracle",
            "sample": main["sample"] + " of " + model + ", %.1f s" % main["seconds"],
            "single_core": runs.get("one"), "build": "gcc -O3 -march=native -fopenmp (%s)" % os.path.basename(lib),
            "host": host}


def batch_comparison() -> dict:
    """64 mixed planning instances submitted at once: one plan per launch vs
    shared launches.  Latency of a plan = completion - submission."""
    from paper_2306_01301_amd import scenes, serving, sizing

    reqs = scenes.batch_64()
    updates = sum(sizing.pose_updates(s.nx, s.nt, s.n_cycles, len(s.schedule)) for s in reqs)
    serving.run_batched(reqs[:8])  # warm-up
    serving.run_single(reqs[:8])
    warm = serving.Server(1 << 60, max_live=8)
    warm.run(reqs[:8], [0.0] * 8)
    warm.close()
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
    from paper_2306_01301_amd import scenes, serving

    pool = scenes.serving_requests(count=args.requests)
    budget = int(args.serve_budget_gib * (1 << 30))
    rates = [float(r) for r in args.rates.split(",") if r]
    warm = serving.Server(budget, max_live=64)
    warm.run(pool[:4], [0.0] * 4)
    warm.close()
    per_rate = []
    for rate in rates:
        # a window of `seconds` of arrivals (at most --max-requests), cycling the pool of distinct requests
        count = len(pool) if args.seconds <= 0 else min(args.max_requests, max(len(pool), int(args.seconds * rate)))
        reqs = [pool[k % len(pool)] for k in range(count)]
        arr = scenes.poisson_arrivals(1306 + int(rate), rate, len(reqs))
        srv = serving.Server(budget, max_live=64)
        res = srv.run(reqs, arr)
        srv.close()
        s = serving.latency_summary(res)
        s["rate"] = rate
        s["requests"] = len(reqs)
        s["peak_admitted_bytes"] = srv.peak_held
        s["admission_waits"] = srv.admission_waits
        print(json.dumps({"rate": rate, "server": s}), file=sys.stderr, flush=True)
        s["one_plan_at_a_time"] = serving.latency_summary(serving.run_fifo(reqs, arr))
        per_rate.append(s)
        print(json.dumps({"rate": rate, "fifo": s["one_plan_at_a_time"]}), file=sys.stderr, flush=True)
    best = max(per_rate, key=lambda s: s["plans_per_s"] or 0)
    out = {"metric": METRIC, "value": best["plans_per_s"], "unit": "plans/s", "n_gpus": 1, "steps": len(rates),
           "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u32", "data": "synthetic",
           "config": {"workload": "serving_requests", "distinct_requests": len(pool), "seconds_per_rate": args.seconds,
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


def bench_batch_modes(args) -> int:
    """batch_64 once in one mode (--mode batched|continuous|single), after a
    warm-up and a marker kernel (a fill of 7777 words), for kernel traces:
    python -m paper_2306_01301_amd.profsum gaps DIR reads the trace after the
    marker."""
    import torch

    from paper_2306_01301_amd import scenes, serving

    reqs = scenes.batch_64()
    serving.run_batched(reqs[:8])
    serving.run_single(reqs[:8])
    warm = serving.Server(1 << 60, max_live=8)
    warm.run(reqs[:8], [0.0] * 8)
    warm.close()
    torch.cuda.synchronize()
    torch.full((7777,), 7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.mode == "batched":
        res = serving.run_batched(reqs)
    elif args.mode == "single":
        res = serving.run_single(reqs)
    else:
        srv = serving.Server(1 << 60, max_live=len(reqs))
        res = srv.run(reqs, [0.0] * len(reqs))
        srv.close()
    torch.cuda.synchronize()
    print(json.dumps({"workload": "batch_64", "mode": args.mode, "wall_ms": (time.perf_counter() - t0) * 1e3,
                      **serving.latency_summary(res)}), flush=True)
    return 0


def other_workloads(reps: int = 20) -> dict:
    """The paper-shaped small workloads through the plain entry points
    (render_cspace, sweep_n_turns, extract_path) on a planner made once:
    median time per whole plan and the sweep throughput."""
    import torch

    from paper_2306_01301_amd import planner, scenes, sizing

    out = {}
    for name in ("parking_256", "plain_64"):
        sc = scenes.WORKLOADS[name]()
        p = planner.planner_for(sc)
        image = torch.from_numpy(np.ascontiguousarray(sc.image)).cuda()

        def plan():
            p.render(image, sc.vehicle)
            p.sweep(sc.start, sc.n_cycles)
            return p.extract(sc.goal, sc.goal_radius, sc.w_xy, sc.w_t)

        for _ in range(3):
            plan()
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            path = plan()  # extract synchronises
            times.append(time.perf_counter() - t0)
        ms = 1000.0 * float(np.median(times))
        updates = sizing.pose_updates(sc.nx, sc.nt, sc.n_cycles, len(sc.schedule))
        out[name] = {"grid": [sc.nx, sc.nx, sc.nt], "n_cycles": sc.n_cycles, "ms_per_plan": ms,
                     "plans_per_s": 1000.0 / ms, "pose_updates_per_s": updates / (ms * 1e-3),
                     "plan_maneuvers": len(path.steps), "reps": reps}
        p.close()
    return out


def serving_block(rates, count: int, budget: int) -> dict:
    """Continuous batching under Poisson arrivals of the mixed serving
    requests, against the same arrivals served one plan at a time, per
    rate; admission by the 25 B/pose formula against `budget` bytes."""
    from paper_2306_01301_amd import scenes, serving

    reqs = scenes.serving_requests(count=count)
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
        s["peak_admitted_bytes"] = srv.peak_held
        s["admission_waits"] = srv.admission_waits
        s["one_plan_at_a_time"] = serving.latency_summary(serving.run_fifo(reqs, arr))
        per_rate.append(s)
        print(json.dumps({"serving_rate": rate, "p50_ms": s["p50_ms"], "p99_ms": s["p99_ms"],
                          "fifo_p99_ms": s["one_plan_at_a_time"]["p99_ms"]}), file=sys.stderr, flush=True)
    return {"workload": "serving_requests", "requests_per_rate": len(reqs), "hbm_budget_bytes": budget,
            "admission": "25 B/pose (3 vertices x 2 gears x 4 B + 1 B collision)", "rates": per_rate}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="maze_512")
    ap.add_argument("--cpu-cycles", type=int, default=20,
                    help="oracle cycles timed on all host CPUs for cpu_baseline (0: skip the CPU baseline)")
    ap.add_argument("--cpu-cycles-one", type=int, default=2, help="oracle cycles timed on one core")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain device copy of 1 GiB (counter calibration)")
    ap.add_argument("--skip-batch", action="store_true", help="skip the batched-vs-single comparison")
    ap.add_argument("--skip-serving", action="store_true", help="skip the serving block")
    ap.add_argument("--skip-other", action="store_true", help="skip the parking_256 and plain_64 lines")
    ap.add_argument("--skip-check", action="store_true", help="skip the check against sweep_n_turns")
    ap.add_argument("--serve-rates", default="20,100", help="serving block: Poisson rates in plans/s")
    ap.add_argument("--serve-requests", type=int, default=300, help="serving block: requests per rate")
    ap.add_argument("--serve-budget-gib", type=float, default=16.0, help="serving block: admission budget")
    ap.add_argument("--mode", default="batched", help="batch_64 workload: batched, continuous or single")
    ap.add_argument("--rates", default="10,20,50,100,200,500",
                    help="serving workload: Poisson arrival rates in plans/s")
    ap.add_argument("--requests", type=int, default=300, help="serving workload: distinct requests (the pool)")
    ap.add_argument("--seconds", type=float, default=0.0,
                    help="serving workload: seconds of arrivals per rate, cycling the pool (0: the pool once)")
    ap.add_argument("--max-requests", type=int, default=1200, help="serving workload: cap on requests per rate")
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
    if args.workload == "batch_64":
        return bench_batch_modes(args)
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
    family = p.tables()["I"]
    n_planes = {"straight_x": int(np.sum(family == 0)), "straight_y": int(np.sum(family == 1))}
    N2 = sc.nx * sc.nx

    def one_plan(events):
        """One step.  events: list to append (tag, event) pairs to, or None.
        A straight pass is its two kernels (y-major planes, then x-major
        planes), with an event after each."""
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
        for a, b in passes:  # the passes sweep_n_turns runs
            if kernel_kind(a, b) == "straight":
                p.sweep_straight_family(a, 1)
                mark("straight_y")
                p.sweep_straight_family(a, 0)
                mark("straight_x")
            else:
                p.sweep_pass(a, b)
                mark(kernel_kind(a, b))
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

    # per-stage and per-kernel durations from the events (plan's stream)
    stage = {"render": [], "init": [], "sweeps": [], "extract": []}
    kinds = {k: [] for k in KERNELS}
    for ev in step_events:
        t = {}
        sweeps = 0.0
        for (_, ea), (tag, eb) in zip(ev[:-1], ev[1:]):
            dt = ea.elapsed_time(eb)
            if tag in ("render", "init", "extract"):
                t[tag] = dt
            else:
                sweeps += dt
                kinds[tag].append(dt)
        for k in ("render", "init", "extract"):
            stage[k].append(t[k])
        stage["sweeps"].append(sweeps)

    check = None
    if not args.skip_check:
        # the timed steps drove the passes one by one: the last step's value
        # volume and plan must equal what sweep_n_turns (captured cycle
        # graphs) leaves, which the parity tests compare with the oracle
        timed_V = p.value.clone()
        p.sweep(sc.start, sc.n_cycles)
        ref = p.extract(sc.goal, sc.goal_radius, sc.w_xy, sc.w_t)
        same_V = bool(torch.equal(p.value, timed_V))
        same_plan = (path.best, path.value, path.score, path.steps) == (ref.best, ref.value, ref.score, ref.steps)
        if not (same_V and same_plan):
            print("bench: the timed passes disagree with sweep_n_turns (value volume equal: %s, plan equal: %s)"
                  % (same_V, same_plan), file=sys.stderr)
            return 1
        check = "value volume and plan of the timed passes equal to sweep_n_turns"
        del timed_V

    updates = sizing.pose_updates(sc.nx, sc.nt, sc.n_cycles, n_sched)
    ms_per_step = 1000.0 * wall / args.steps
    traffic = measured_traffic()
    per_kernel = {}
    alg_bytes_step = 0.0
    measured_bytes_step = 0.0
    for k, v in kinds.items():
        if not v:
            continue
        avg = float(np.mean(v))
        planes = n_planes.get(k, sc.nt)
        nbytes = BYTES_PER_UPDATE * N2 * planes  # read V, read code, write V once per pose of the launch
        per_step = len(v) // args.steps
        alg_bytes_step += nbytes * per_step
        gbs = nbytes / (avg * 1e-3) / 1e9
        ups = 2 if k == "fused_turn" else 1
        tr = traffic.get(k)
        measured_bytes_step = (measured_bytes_step + tr * per_step) if (tr and measured_bytes_step is not None) else None
        per_kernel[k] = {"kernel": KERNELS[k], "launches_per_step": per_step, "avg_us": avg * 1e3,
                         "ms_per_step": float(np.sum(v)) / args.steps, "planes": planes,
                         "bytes_per_launch": nbytes, "GB_per_s": gbs, "frac_algorithmic": gbs / HBM_PEAK_GBS,
                         "updates_per_pose": ups, "frac_update_equivalent": ups * gbs / HBM_PEAK_GBS,
                         "traffic_bytes_per_launch": tr, "traffic_ratio": (tr / nbytes) if tr else None,
                         "frac_measured": (tr / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS) if tr else None}
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_per_step"])
    sweep_ms = float(np.median(stage["sweeps"]))
    sweep_sum_ms = float(np.mean(stage["sweeps"]))
    lat_ms = np.array(lat) * 1000.0
    d = per_kernel[dom]
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
        "check": check,
        "roofline": {"kernel": d["kernel"], "bound": "hbm", "achieved": d["GB_per_s"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": d["frac_algorithmic"], "traffic": d["traffic_bytes_per_launch"],
                     "bytes_per_launch_algorithmic": d["bytes_per_launch"], "avg_launch_us": d["avg_us"],
                     "launches_timed": len(kinds[dom]),
                     "frac_reading": "algorithmic: 9 B per pose per launch (read the value and the code, write "
                                     "the value); the kernels do not store values that stayed the same, so "
                                     "the bytes they move (traffic, from the counters) are fewer; a fused turn "
                                     "launch relaxes every pose twice for the 9 B",
                     "kernels": per_kernel,
                     "whole_sweep": {"ms": sweep_sum_ms,
                                     "algorithmic_bytes": alg_bytes_step,
                                     "frac_algorithmic": alg_bytes_step / (sweep_sum_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                     "measured_bytes": measured_bytes_step,
                                     "frac_measured": (measured_bytes_step / (sweep_sum_ms * 1e-3) / 1e9
                                                       / HBM_PEAK_GBS) if measured_bytes_step else None,
                                     "update_equivalent_bytes": BYTES_PER_UPDATE * updates,
                                     "frac_update_equivalent": BYTES_PER_UPDATE * updates / (sweep_sum_ms * 1e-3)
                                     / 1e9 / HBM_PEAK_GBS}},
    }
    p.close()
    if not args.skip_other:
        out["other_workloads"] = other_workloads()
    if not args.skip_batch:
        out["latency_ms"]["batch_64"] = batch_comparison()
    if not args.skip_serving:
        rates = [float(r) for r in args.serve_rates.split(",") if r]
        out["serving"] = serving_block(rates, args.serve_requests, int(args.serve_budget_gib * (1 << 30)))
    if args.cpu_cycles > 0:
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_cycles, args.cpu_cycles_one)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
