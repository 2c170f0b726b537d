"""Many planning requests on one GPU: one plan per launch, one batch, and a
continuous-batching server.

* `run_single`: requests one after another, each through the single-plan
  entry points (render_cspace, sweep_n_turns, extract_path).
* `run_batched`: all requests through shared launches (batch_render,
  batch_sweep, batch_extract).
* `Server`: requests arrive over time (e.g. Poisson); a request is admitted
  when its HBM footprint fits the budget, its map and volumes then stay on
  the device until it completes.  Every tick advances every admitted plan by
  a number of sweeps inversely proportional to its size (one batch_advance
  call, all live plans in shared launches); plans that finish their
  sweeps are extracted together and release their memory, and requests that
  arrived meanwhile are admitted at the next tick.

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
    done: int = 0
    per_tick: int = 1
    footprint: int = 0


class Server:
    """Continuous batching over requests that arrive over time."""

    def __init__(self, hbm_budget: int, max_live: int = 64, rule: str = "formula", digests: bool = False):
        self.budget = int(hbm_budget)
        self.max_live = int(max_live)
        self.rule = rule
        self.digests = digests
        self.batch = P.Batch(max_live)

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
                    break
                pending.pop(0)
                held += need
                pl = P.planner_for(sc)
                img = torch.from_numpy(np.ascontiguousarray(sc.image)).cuda()
                fresh.append(_Live(k, sc, pl, img, sc.n_cycles * len(sc.schedule), footprint=need))
                results[k].admitted = time.perf_counter() - t0
            if fresh:
                self.batch.render([f.planner for f in fresh], [f.image for f in fresh], [f.scene.vehicle for f in fresh])
                self.batch.init([f.planner for f in fresh], [f.scene.start for f in fresh])
                live.extend(fresh)
            if not live:
                # idle until the next arrival
                wait = results[pending[0]].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
                continue
            # sweeps per tick: inversely proportional to the plan's size
            biggest = max(l.scene.n_poses for l in live)
            for l in live:
                l.per_tick = max(1, min(l.total - l.done, int(round(biggest / l.scene.n_poses))))
            self.batch.advance([l.planner for l in live], [l.done for l in live], [l.per_tick for l in live])
            for l in live:
                l.done += l.per_tick
            finished = [l for l in live if l.done >= l.total]
            if finished:
                paths = self.batch.extract([l.planner for l in finished], [l.scene.goal for l in finished],
                                           [l.scene.goal_radius for l in finished], [l.scene.w_xy for l in finished],
                                           [l.scene.w_t for l in finished])
                t = time.perf_counter() - t0
                for l, path in zip(finished, paths):
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
        self.batch.close()


def latency_summary(results: Sequence[Result]) -> dict:
    lat = np.array([r.latency for r in results]) * 1000.0
    span = max(r.finished for r in results) - min(r.arrival for r in results)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "plans_per_s": len(results) / span if span > 0 else None,
            "n": len(results), "unreached": int(sum(1 for r in results if r.status != 0))}
