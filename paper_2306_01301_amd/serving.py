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
  the device until it completes.  Small and large plans run in two classes
  on two streams so their launches overlap; within a class every tick
  advances every admitted plan by a number of sweeps inversely proportional
  to its size (one batch_advance call, shared launches); plans that finish
  their sweeps are extracted together and release their memory, and
  requests that arrived meanwhile are admitted at the next tick.

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
    total: int
    cls: int = 0
    done: int = 0
    per_tick: int = 1
    footprint: int = 0


LARGE_POSES = 1 << 25  # plans at least this large go to the large class
LARGE_AT_ONCE = 1      # large plans advanced per tick (1: shortest remaining work first, one at a time)


class Server:
    """Continuous batching over requests that arrive over time.

    Plans are split into two size classes, each with its own stream and
    batch, so that the many short passes of small plans run on the GPU at
    the same time as the long passes of large plans instead of waiting
    between them.  Every tick advances each live small plan, and the large
    plan(s) with the least remaining work (LARGE_AT_ONCE), by a number of
    passes inversely proportional to its size within its class (one
    batch_advance call per class); finished plans are extracted together and
    release their memory, and requests that arrived meanwhile are admitted at
    the next tick."""

    def __init__(self, hbm_budget: int, max_live: int = 64, rule: str = "formula", digests: bool = False):
        self.budget = int(hbm_budget)
        self.max_live = int(max_live)
        self.rule = rule
        self.digests = digests
        self.streams = [torch.cuda.Stream(), torch.cuda.Stream()]  # default priority
        self.batches = [P.Batch(max_live, stream=st) for st in self.streams]
        self.peak_held = 0        # largest admitted footprint at once (bytes)
        self.admission_waits = 0  # ticks on which an arrived request waited for memory

    def run(self, scs: Sequence, arrivals: Sequence[float]) -> List[Result]:
        order = np.argsort(np.asarray(arrivals), kind="stable")
        results = [Result(sc.name, float(a)) for sc, a in zip(scs, arrivals)]
        pending = [int(k) for k in order]
        live: List[_Live] = []
        held = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while pending or live:
            now = time.perf_counter() - t0
            # admit arrived requests while memory and slots allow (in arrival order)
            fresh: List[_Live] = []
            while pending and results[pending[0]].arrival <= now and len(live) + len(fresh) < self.max_live:
                k = pending[0]
                sc = scs[k]
                need = footprint_bytes(sc, self.rule)
                if held + need > self.budget and (live or fresh):
                    self.admission_waits += 1
                    break
                pending.pop(0)
                held += need
                self.peak_held = max(self.peak_held, held)
                cls = 1 if sc.n_poses >= LARGE_POSES else 0
                st = self.streams[cls]
                pl = P.planner_for(sc, stream=st)
                with torch.cuda.stream(st):
                    img = torch.from_numpy(np.ascontiguousarray(sc.image)).cuda()
                fresh.append(_Live(k, sc, pl, img, sc.n_cycles * len(sc.schedule), cls=cls, footprint=need))
                results[k].admitted = time.perf_counter() - t0
            for cls in (0, 1):
                new = [f for f in fresh if f.cls == cls]
                if new:
                    b = self.batches[cls]
                    b.render([f.planner for f in new], [f.image for f in new], [f.scene.vehicle for f in new])
                    b.init([f.planner for f in new], [f.scene.start for f in new])
            live.extend(fresh)
            if not live:
                # idle until the next arrival
                wait = results[pending[0]].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
                continue
            finished: List[_Live] = []
            for cls in (0, 1):
                mine = [l for l in live if l.cls == cls]
                if cls == 1:
                    # large plans: the ones with the least remaining work first
                    # (shortest remaining work keeps the mean latency low),
                    # LARGE_AT_ONCE at a time so they do not slow each other down
                    mine.sort(key=lambda l: (l.total - l.done) * l.scene.n_poses)
                    mine = mine[:LARGE_AT_ONCE]
                if not mine:
                    continue
                # passes per tick: inversely proportional to the plan's size;
                # a tick ends on a pass boundary so that turn pairs stay fused
                biggest = max(l.scene.n_poses for l in mine)
                for l in mine:
                    want = max(1, int(round(biggest / l.scene.n_poses)))
                    passes = P.schedule_passes(l.scene.schedule, l.done, l.total - l.done)[:want]
                    l.per_tick = sum(1 if b < 0 else 2 for _, b in passes)
                self.batches[cls].advance([l.planner for l in mine], [l.done for l in mine],
                                          [l.per_tick for l in mine])
                for l in mine:
                    l.done += l.per_tick
                finished += [l for l in mine if l.done >= l.total]
            for cls in (0, 1):
                done = [l for l in finished if l.cls == cls]
                if not done:
                    continue
                paths = self.batches[cls].extract([l.planner for l in done], [l.scene.goal for l in done],
                                                  [l.scene.goal_radius for l in done], [l.scene.w_xy for l in done],
                                                  [l.scene.w_t for l in done])
                t = time.perf_counter() - t0
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
                    held -= l.footprint
            live = [l for l in live if l.done < l.total]
        return results

    def close(self) -> None:
        for b in self.batches:
            b.close()


def latency_summary(results: Sequence[Result]) -> dict:
    lat = np.array([r.latency for r in results]) * 1000.0
    span = max(r.finished for r in results) - min(r.arrival for r in results)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "plans_per_s": len(results) / span if span > 0 else None,
            "n": len(results), "unreached": int(sum(1 for r in results if r.status != 0))}
