"""Many planning requests on one GPU: one plan per launch, one batch, and a
continuous-batching server.

* `run_single`: requests one after another, each through the single-plan
  entry points (render_cspace, sweep_n_turns, extract_path).
* `run_batched`: all requests through shared launches (batch_render,
  batch_sweep, batch_extract).
* `run_fifo`: requests that arrive over time served one at a time in
  arrival order through the single-plan entry points.
* `Server`: requests arrive over time (e.g. Poisson); a request is admitted
  when its HBM footprint fits the budget, its map and volumes then stay on
  the device until it completes.  Admission (plan, image, rendering, init),
  sweeps (shared launches of the live plans picked per tick, shortest
  remaining work first with aging) and extraction run on three streams, so
  neither admission nor extraction waits for queued sweeps.

Host code only (scheduling and bookkeeping); all planning work runs in the
HIP library.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import planner as P
from . import sizing


@dataclass
class Result:
    name: str
    arrival: float          # s, relative to the run's start
    admitted: float = 0.0
    finished: float = 0.0
    status: int = 0         # 0 or an NHP_E* code
    path: Optional[P.Path] = None
    value_digest: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def footprint_bytes(scene, rule: str = "formula") -> int:
    """HBM a request holds while admitted: `formula` = 3 vertices x 2 gears x
    4 B per pose plus the 1 B collision volume; `real` = this library's
    workspace (4 B value + 1 B obstacle code per pose plus tables)."""
    if rule == "formula":
        return sizing.admission_bytes(scene.nx, scene.nt)
    return P.workspace_bytes(P.make_params(scene.nx, scene.nt, scene.R, scene.ct, scene.gear, scene.schedule,
                                           scene.half_cell)) + scene.nx * scene.nx


def _digest(p: P.Planner) -> str:
    import hashlib

    return hashlib.sha1(p.value_numpy().tobytes()).hexdigest()


def run_single(scs: Sequence, digests: bool = False) -> List[Result]:
    """One plan at a time (all submitted at t = 0)."""
    out = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sc in scs:
        r = Result(sc.name, 0.0)
        p = P.planner_for(sc)
        img = torch.from_numpy(np.ascontiguousarray(sc.image)).cuda()
        p.render(img, sc.vehicle)
        p.sweep(sc.start, sc.n_cycles)
        try:
            r.path = p.extract(sc.goal, sc.goal_radius, sc.w_xy, sc.w_t, cap=512)
        except P.NhpError as e:
            r.status = e.rc
        r.finished = time.perf_counter() - t0
        if digests:
            r.value_digest = _digest(p)
        p.close()
        out.append(r)
    return out


def run_fifo(scs: Sequence, arrivals: Sequence[float]) -> List[Result]:
    """One plan at a time in arrival order through the single-plan entry
    points (the baseline for the server: no sharing of launches)."""
    order = np.argsort(np.asarray(arrivals), kind="stable")
    results = [Result(sc.name, float(a)) for sc, a in zip(scs, arrivals)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in order:
        k = int(k)
        wait = results[k].arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        sc = scs[k]
        results[k].admitted = time.perf_counter() - t0
        p = P.planner_for(sc)
        img = torch.from_numpy(np.ascontiguousarray(sc.image)).cuda()
        p.render(img, sc.vehicle)
        p.sweep(sc.start, sc.n_cycles)
        try:
            results[k].path = p.extract(sc.goal, sc.goal_radius, sc.w_xy, sc.w_t, cap=512)
        except P.NhpError as e:
            results[k].status = e.rc
        results[k].finished = time.perf_counter() - t0
        p.close()
    return results


def run_batched(scs: Sequence, digests: bool = False) -> List[Result]:
    """All plans in shared launches (all submitted at t = 0)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    planners = [P.planner_for(sc) for sc in scs]
    images = [torch.from_numpy(np.ascontiguousarray(sc.image)).cuda() for sc in scs]
    b = P.Batch(len(scs))
    b.render(planners, images, [sc.vehicle for sc in scs])
    b.sweep(planners, [sc.start for sc in scs], [sc.n_cycles for sc in scs])
    paths = b.extract(planners, [sc.goal for sc in scs], [sc.goal_radius for sc in scs],
                      [sc.w_xy for sc in scs], [sc.w_t for sc in scs])
    t1 = time.perf_counter() - t0
    out = []
    for sc, p, path in zip(scs, planners, paths):
        r = Result(sc.name, 0.0, finished=t1)
        if isinstance(path, int):
            r.status = path
        else:
            r.path = path
        if digests:
            r.value_digest = _digest(p)
        out.append(r)
    b.close()
    for p in planners:
        p.close()
    return out


@dataclass
class _Live:
    k: int
    scene: object
    planner: P.Planner
    image: torch.Tensor
    total: int              # sweeps of the plan
    arrival: float
    done: int = 0           # sweeps enqueued so far
    footprint: int = 0
    finish_event: Optional[torch.cuda.Event] = None  # a plan with no sweeps: the event it was handed over with

    @property
    def remaining_updates(self) -> int:
        return (self.total - self.done) * self.scene.n_poses


# Scheduling of a tick (see tick_plan); the autotuner's measured choice in
# tuning.json replaces the first three.
FILL_POSES = 64 << 20    # poses a tick's passes cover together before it stops adding plans
TICK_POSES = 1 << 30     # pose updates each selected plan gets per tick (at least one pass)
ADMIT_PER_TICK = 4       # requests per hand-over to the admission thread
AGING = 1.0              # seconds of expected work a second of waiting is worth
UPDATE_RATE = 6.0e11     # pose updates per second of the sweep kernels, for the expected-work estimate
MAX_QUEUED_TICKS = 2     # ticks enqueued ahead of the GPU
_tuned = P.load_tuning().get("server", {})
FILL_POSES = int(_tuned.get("fill_poses", FILL_POSES))
TICK_POSES = int(_tuned.get("tick_poses", TICK_POSES))
ADMIT_PER_TICK = int(_tuned.get("admit_per_tick", ADMIT_PER_TICK))


def tick_plan(live: Sequence[_Live], now: float, fill_poses: int = FILL_POSES, tick_poses: int = TICK_POSES,
              aging: float = AGING, rate: float = UPDATE_RATE):
    """Which live plans advance this tick, and by how many sweeps.

    Plans are taken in order of expected remaining work minus `aging` times
    their time in the system (shortest remaining work first, with older
    requests moving up so that a large request is not passed over
    indefinitely), until their passes together cover `fill_poses` poses (so
    every shared launch has enough tiles to fill the GPU).  Each selected
    plan runs whole passes worth about `tick_poses` pose updates (at least
    one pass; a tick ends on a pass boundary so turn pairs stay fused).
    Returns [(plan, sweeps)]."""
    runnable = [l for l in live if l.done < l.total]
    runnable.sort(key=lambda l: (l.remaining_updates / rate - aging * (now - l.arrival), l.arrival, l.k))
    out, covered = [], 0
    for l in runnable:
        if covered >= fill_poses:
            break
        want = max(1, int(round(tick_poses / l.scene.n_poses)))
        passes = P.schedule_passes(l.scene.schedule, l.done, l.total - l.done)[:want]
        out.append((l, sum(1 if b < 0 else 2 for _, b in passes)))
        covered += l.scene.n_poses
    return out


class Server:
    """Continuous batching over requests that arrive over time.

    Three streams and two worker threads keep the GPU fed:
      * admission: arrived requests whose HBM footprint fits the budget are
        handed, most urgent first (the tick priority below), to a worker
        thread that makes their plans, uploads their images, renders their
        obstacle volumes and initialises their value volumes on its own
        stream, so neither this host work nor the synchronisations it needs
        hold up the sweeps (the library's calls release the interpreter
        lock while they run).  When no sweeps are running or queued there
        is nothing to overlap, and the scheduling thread admits the requests
        itself, sparing the hand-over;
      * sweeps: each tick, the plans tick_plan picks advance together in
        shared launches (batch_advance); at most MAX_QUEUED_TICKS ticks are
        enqueued ahead of the GPU;
      * extraction: the plans whose last sweeps a tick enqueues go at once
        to a second worker thread, which waits for that tick, runs their
        goal search and back-tracking on the extraction stream and releases
        their plans, so the scheduling thread never waits for an
        extraction.
    Requests that arrive meanwhile are admitted as memory and slots free."""

    def __init__(self, hbm_budget: int, max_live: int = 64, rule: str = "formula", digests: bool = False,
                 fill_poses: int = FILL_POSES, tick_poses: int = TICK_POSES, aging: float = AGING,
                 admit_per_tick: int = ADMIT_PER_TICK):
        self.budget = int(hbm_budget)
        self.max_live = int(max_live)
        self.rule = rule
        self.digests = digests
        self.fill_poses, self.tick_poses, self.aging = int(fill_poses), int(tick_poses), float(aging)
        self.admit_per_tick = int(admit_per_tick)  # requests per hand-over to the admission thread
        self.device = torch.cuda.current_device()
        # default priority for every stream
        self.s_admit, self.s_sweep, self.s_extract = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
        self.b_admit = P.Batch(max_live, stream=self.s_admit)
        self.b_sweep = P.Batch(max_live, stream=self.s_sweep)
        self.b_extract = P.Batch(max_live, stream=self.s_extract)
        self.peak_held = 0        # largest admitted footprint at once (bytes)
        self.admission_waits = 0  # ticks on which an arrived request waited for memory
        self.admitted_inline = 0  # requests admitted by the scheduling thread (sweeps idle)
        self.ticks = 0
        self.host_s = {"admit": 0.0, "tick": 0.0, "wait": 0.0}  # scheduling-thread host time per phase

    def _admit(self, job) -> tuple:
        """Plans, images, rendering and init of requests [(k, scene, arrival,
        footprint)] on the admission stream; returns (fresh plans, event)."""
        fresh = []
        with torch.cuda.stream(self.s_admit):
            for k, sc, arrival, need in job:
                pl = P.planner_for(sc, stream=self.s_admit)
                img = torch.from_numpy(np.ascontiguousarray(sc.image)).cuda()
                fresh.append(_Live(k, sc, pl, img, sc.n_cycles * len(sc.schedule), arrival, footprint=need))
            planners = [f.planner for f in fresh]
            self.b_admit.render(planners, [f.image for f in fresh], [f.scene.vehicle for f in fresh])
            self.b_admit.init(planners, [f.scene.start for f in fresh])
            ready = torch.cuda.Event()
            ready.record(self.s_admit)
        return fresh, ready

    def _admission(self, inbox: "queue.Queue", outbox: "queue.Queue") -> None:
        """Worker thread: admission of handed-over requests."""
        torch.cuda.set_device(self.device)
        while True:
            job = inbox.get()
            if job is None:
                return
            try:
                outbox.put(self._admit(job))
            except BaseException as e:  # handed to the main thread, which raises it
                outbox.put((e, None))

    def _extraction(self, inbox: "queue.Queue", outbox: "queue.Queue", results: List[Result], t0: list) -> None:
        """Worker thread: goal search and back-tracking of the plans whose
        last sweeps one tick enqueued (handed over together with that tick's
        event), then their release.  Posts the finished plans back."""
        torch.cuda.set_device(self.device)
        while True:
            group = inbox.get()
            if group is None:
                return
            try:
                done, ev = group
                self.s_extract.wait_event(ev)
                for l in done:
                    l.planner.set_stream(self.s_extract)  # its own work (digest, destroy) waits on this stream
                if len(done) == 1:
                    # one plan: extract_path, whose back-tracking spreads each step over one
                    # workgroup per scheduled maneuver (a batch gives each plan one workgroup)
                    l = done[0]
                    try:
                        paths = [l.planner.extract(l.scene.goal, l.scene.goal_radius, l.scene.w_xy,
                                                   l.scene.w_t, cap=512)]
                    except P.NhpError as e:
                        paths = [e.rc]
                else:
                    paths = self.b_extract.extract([l.planner for l in done], [l.scene.goal for l in done],
                                                   [l.scene.goal_radius for l in done],
                                                   [l.scene.w_xy for l in done], [l.scene.w_t for l in done])
                t = time.perf_counter() - t0[0]
                for l, path in zip(done, paths):
                    r = results[l.k]
                    r.finished = t
                    if isinstance(path, int):
                        r.status = path
                    else:
                        r.path = path
                    if self.digests:
                        r.value_digest = _digest(l.planner)
                    l.planner.close()
                outbox.put(done)
            except BaseException as e:  # handed to the main thread, which raises it
                outbox.put(e)

    def run(self, scs: Sequence, arrivals: Sequence[float]) -> List[Result]:
        import queue
        import threading

        results = [Result(sc.name, float(a)) for sc, a in zip(scs, arrivals)]
        pending = [int(k) for k in np.argsort(np.asarray(arrivals), kind="stable")]
        work = {k: sizing.pose_updates(scs[k].nx, scs[k].nt, scs[k].n_cycles, len(scs[k].schedule)) / UPDATE_RATE
                for k in pending}
        live: List[_Live] = []       # admitted and ready: sweeps still to enqueue, or extraction still to end
        admitting = 0                # handed to the admission thread, not back yet
        extracting = 0               # plans handed to the extraction thread, not back yet
        queued: List[torch.cuda.Event] = []  # one per enqueued tick
        held = 0
        inbox, outbox = queue.Queue(), queue.Queue()
        x_in, x_out = queue.Queue(), queue.Queue()
        t0_box = [0.0]  # the run's start, for the extraction thread's finish times
        worker = threading.Thread(target=self._admission, args=(inbox, outbox), daemon=True)
        extractor = threading.Thread(target=self._extraction, args=(x_in, x_out, results, t0_box), daemon=True)
        worker.start()
        extractor.start()
        torch.cuda.synchronize()
        t0 = t0_box[0] = time.perf_counter()
        clock = time.perf_counter

        def take(fresh, ready):
            self.s_sweep.wait_event(ready)  # the sweeps of these plans come after their init
            for f in fresh:
                f.planner.set_stream(self.s_sweep)
            live.extend(fresh)

        try:
            while pending or live or admitting:
                now = clock() - t0
                h0 = clock()
                # ---- plans whose extraction has ended release their memory ----
                freed = False
                while True:
                    try:
                        done = x_out.get_nowait()
                    except queue.Empty:
                        break
                    if isinstance(done, BaseException):
                        raise done
                    freed = True
                    extracting -= len(done)
                    held -= sum(l.footprint for l in done)
                    gone = set(id(l) for l in done)
                    live = [l for l in live if id(l) not in gone]
                # ---- admission: arrived requests, most urgent first (expected
                # work minus aging), memory and slots permitting ----
                arrived = [k for k in pending if results[k].arrival <= now]
                arrived.sort(key=lambda k: (work[k] - self.aging * (now - results[k].arrival), results[k].arrival, k))
                job = []
                if admitting < 2 * self.admit_per_tick:
                    for k in arrived:
                        if len(live) + admitting + len(job) >= self.max_live or len(job) >= self.admit_per_tick:
                            break
                        sc = scs[k]
                        need = footprint_bytes(sc, self.rule)
                        if held + need > self.budget and (live or admitting or job):
                            self.admission_waits += 1
                            break
                        pending.remove(k)
                        held += need
                        self.peak_held = max(self.peak_held, held)
                        job.append((k, sc, results[k].arrival, need))
                        results[k].admitted = clock() - t0
                queued = [e for e in queued if not e.query()]
                got = False
                if job:
                    if not queued and admitting == 0 and all(l.done >= l.total for l in live):
                        # no sweeps to overlap with: admit here, without the hand-over
                        take(*self._admit(job))
                        self.admitted_inline += len(job)
                        got = True
                    else:
                        inbox.put(job)
                        admitting += len(job)
                while True:
                    try:
                        fresh, ready = outbox.get_nowait()
                    except queue.Empty:
                        break
                    if isinstance(fresh, BaseException):
                        raise fresh
                    got = True
                    take(fresh, ready)
                    admitting -= len(fresh)
                h1 = clock()
                self.host_s["admit"] += h1 - h0
                # ---- one tick of sweeps ----
                picked = tick_plan(live, now, self.fill_poses, self.tick_poses, self.aging) \
                    if len(queued) < MAX_QUEUED_TICKS else []
                if picked:
                    self.b_sweep.advance([l.planner for l, _ in picked], [l.done for l, _ in picked],
                                         [n for _, n in picked])
                    ev = torch.cuda.Event()
                    ev.record(self.s_sweep)
                    queued.append(ev)
                    self.ticks += 1
                    finishing = []
                    for l, n in picked:
                        l.done += n
                        if l.done >= l.total:
                            finishing.append(l)
                    if finishing:
                        # extraction follows this tick on the extraction thread
                        x_in.put((finishing, ev))
                        extracting += len(finishing)
                # plans admitted with no sweeps to run go straight to extraction
                empty = [l for l in live if l.total == 0 and l.finish_event is None]
                if empty:
                    ev = torch.cuda.Event()
                    ev.record(self.s_sweep)
                    for l in empty:
                        l.finish_event = ev
                    x_in.put((empty, ev))
                    extracting += len(empty)
                h2 = clock()
                self.host_s["tick"] += h2 - h1
                if not picked and not got and not job and not freed and not empty:
                    if queued:
                        queued[0].synchronize()  # nothing to do until the oldest enqueued tick completes
                    elif admitting:
                        try:  # wait for the admission thread
                            outbox.put(outbox.get(timeout=0.005))
                        except queue.Empty:
                            pass
                    elif extracting:
                        try:  # wait for the extraction thread
                            x_out.put(x_out.get(timeout=0.005))
                        except queue.Empty:
                            pass
                    elif pending:
                        wait = min(results[k].arrival for k in pending) - (clock() - t0)
                        if wait > 0:
                            time.sleep(min(wait, 0.005))
                    self.host_s["wait"] += clock() - h2
        finally:
            inbox.put(None)
            x_in.put(None)
            worker.join()
            extractor.join()
        return results

    def close(self) -> None:
        for b in (self.b_admit, self.b_sweep, self.b_extract):
            b.close()


def latency_summary(results: Sequence[Result]) -> dict:
    lat = np.array([r.latency for r in results]) * 1000.0
    span = max(r.finished for r in results) - min(r.arrival for r in results)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "plans_per_s": len(results) / span if span > 0 else None,
            "n": len(results), "unreached": int(sum(1 for r in results if r.status != 0))}
