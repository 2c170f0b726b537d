"""Autotuner for the sweep kernels' tile and launch shapes and the server's
schedule.

Three stages, each measured with HIP events on the GPU it runs on and
written to tuning.json, which the binding hands to the library when it
loads (and the server reads):

* sections: a sweep workgroup owns 64 curves and splits each curve into
  sections of P steps held by one wave each; every valid P (8, 16, 32 or 64
  with at most 16 sections) gives identical results, the speed differs with
  the curve length, the grid and the chip.  The fastest P per curve length
  (a turn pass plus a straight pass over free space).
* knobs: resident workgroups per compute unit of the row and x-major
  launches, the tile order (XCD-aware or launch order) and the x-major tile
  buffering (nhp_set_knob), as a grid over their values scored on a fused
  turn pass plus a straight pass at 512^3 and at 256^2 x 128.
* server: the continuous-batching tick (poses a tick fills, pose updates per
  plan per tick, requests per hand-over to the admission thread) on 64 mixed
  instances submitted at once: highest plans/s.

    python -m paper_2306_01301_amd.autotune [--stages sections,knobs,server]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import torch

from . import planner as P
from . import scenes


def _time_ms(fn, reps: int = 10) -> float:
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def _time_on(pl, snapshot: torch.Tensor, fn, reps: int = 10) -> float:
    """ms per call of fn, every call starting from the value volume
    `snapshot` (restored before each call, outside the timed region).
    Unchanged values are not stored, so a pass takes longer the more values
    it changes; timing every setting from the same volume keeps the
    comparison fair."""
    st = pl.stream
    evs = []
    with torch.cuda.stream(st):
        pl.value.copy_(snapshot)
        fn()
        for _ in range(reps):
            pl.value.copy_(snapshot)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(st)
            fn()
            b.record(st)
            evs.append((a, b))
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in evs) / reps


def candidates(length: int):
    return [p for p in (8, 16, 32, 64) if (length + p - 1) // p <= 16]


def measure(length: int) -> dict:
    """ms per sweep for each candidate: a turn sweep over curves of this
    length and a straight sweep over lines of this length."""
    turn_nx = 256 if length > 512 else min(512, max(64, length))
    straight_nt = 128
    out = {}
    for p in candidates(length):
        P.set_section_steps(length, p)
        total = 0.0
        for nx, nt, mu in ((turn_nx, length, P.LF), (length, straight_nt, P.SF)):
            sc = scenes.free_space(nx, nt, max(1.0, nt / 8.0), 1).with_(ct=scenes.uniform_ct(8))
            pl = P.planner_for(sc)
            pl.render(torch.zeros((nx, nx), dtype=torch.uint8, device="cuda"), (1, 1, 1))
            pl.sweep(sc.start, 0)
            total += _time_ms(lambda: pl.sweep_one(mu))
            pl.close()
        out[p] = total
    P.set_section_steps(length, 0)
    return out


KNOB_NAMES = {"row_wg_per_cu": 0, "xmajor_wg_per_cu": 1, "tile_order": 2, "xmajor_buffers": 3}
KNOB_GRID = {"row_wg_per_cu": (0, 1, 2), "xmajor_wg_per_cu": (0, 4, 6), "tile_order": (0, 2),
             "xmajor_buffers": (0, 2)}  # 0: the built-in choice (XCD-aware tiles, one band tile buffer)


def set_knobs(values: dict) -> None:
    for name, v in values.items():
        P.set_knob(KNOB_NAMES[name], int(v))


def measure_knobs(reps: int = 10) -> list:
    """ms of a fused turn pass plus a straight pass on a 512^3 and a 256^2 x
    128 free-space volume for every knob setting of KNOB_GRID, each timed
    from the volume one cycle from the start leaves."""
    import itertools

    shapes = []
    for nx, nt in ((512, 512), (256, 128)):
        sc = scenes.free_space(nx, nt, max(1.0, nt / 8.0), 1).with_(ct=scenes.uniform_ct(8))
        pl = P.planner_for(sc)
        pl.render(torch.zeros((nx, nx), dtype=torch.uint8, device="cuda"), (1, 1, 1))
        pl.sweep(sc.start, 1)
        shapes.append(((nx, nt), pl, pl.value.clone()))
    names = list(KNOB_GRID)
    rows = []
    for combo in itertools.product(*(KNOB_GRID[n] for n in names)):
        values = dict(zip(names, combo))
        set_knobs(values)
        ms = {}
        for (nx, nt), pl, snap in shapes:
            ms["%dx%d" % (nx, nt)] = round(
                _time_on(pl, snap, lambda: (pl.sweep_pass(P.RB, P.RF), pl.sweep_one(P.SF)), reps), 4)
        rows.append({"knobs": values, "ms": ms})
        print("knobs %s: %s" % (values, ms), flush=True)
    set_knobs({n: 0 for n in names})
    for _, pl, _ in shapes:
        pl.close()
    return rows


MARGIN = 0.02  # a measured choice replaces the built-in one only when it is at least this much faster


def builtin_section(length: int) -> int:
    """The library's own choice: the smallest power of two in [8, 64] that
    splits the curve into at most 16 sections."""
    P_ = 8
    while P_ < 64 and P_ * 16 < length:
        P_ *= 2
    return P_


def choose_section(length: int, ms: dict) -> int:
    best = min(ms, key=ms.get)
    base = builtin_section(length)
    if base in ms and ms[best] > (1.0 - MARGIN) * ms[base]:
        return base
    return best


def best_knobs(rows: list) -> dict:
    """The setting with the smallest sum of times relative to the built-in
    setting over the shapes, when that sum beats the built-in one by MARGIN
    per shape on average; otherwise the built-in setting (all zeros)."""
    base = next(r["ms"] for r in rows if all(v == 0 for v in r["knobs"].values()))
    score = lambda r: sum(r["ms"][k] / base[k] for k in base)
    best = min(rows, key=score)
    if score(best) > len(base) * (1.0 - MARGIN):
        return {n: 0 for n in best["knobs"]}
    return best["knobs"]


def measure_server(reps: int = 2) -> list:
    """batch_64 (64 mixed instances, all submitted at once) through the
    server for a grid of tick settings: plans/s and p50, best of `reps`."""
    import itertools

    from . import serving

    reqs = scenes.batch_64()
    serving.run_batched(reqs[:8])
    rows = []
    for fill, tick, admit in itertools.product((32 << 20, 64 << 20, 128 << 20), (256 << 20, 1 << 30), (2, 4)):
        runs = []
        for _ in range(reps):
            srv = serving.Server(1 << 60, max_live=len(reqs), fill_poses=fill, tick_poses=tick, admit_per_tick=admit)
            runs.append(serving.latency_summary(srv.run(reqs, [0.0] * len(reqs))))
            srv.close()
        best = max(runs, key=lambda s: s["plans_per_s"])
        row = {"fill_poses": fill, "tick_poses": tick, "admit_per_tick": admit,
               "plans_per_s": round(best["plans_per_s"], 1), "p50_ms": round(best["p50_ms"], 1)}
        rows.append(row)
        print("server %s" % row, flush=True)
    return rows


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--lengths", default="64,72,128,200,256,384,512,1024")
    ap.add_argument("--stages", default="sections,knobs,server")
    ap.add_argument("--out", default=P.TUNING_PATH)
    args = ap.parse_args()
    stages = set(args.stages.split(","))
    torch.cuda.set_device(0)
    P.lib()
    try:
        with open(args.out) as f:
            doc = json.load(f)
    except (OSError, ValueError):
        doc = {}
    doc["device"] = torch.cuda.get_device_name(0)
    if "sections" in stages:
        table, measured = {}, {}
        for length in [int(x) for x in args.lengths.split(",") if x]:
            if length % 8 or length < 16:
                continue
            ms = measure(length)
            best = choose_section(length, ms)
            table[str(length)] = best
            measured[str(length)] = {str(k): round(v, 4) for k, v in ms.items()}
            print("length %4d: %s -> %d" % (length, measured[str(length)], best), flush=True)
        doc["section_steps"] = table
        doc["measured_ms_turn_plus_straight"] = measured
        P.apply_tuning_table(table)
    if "knobs" in stages:
        rows = measure_knobs()
        doc["knobs"] = best_knobs(rows)
        doc["measured_knobs_ms_fused_turn_plus_straight"] = rows
        print("knobs -> %s" % doc["knobs"], flush=True)
        set_knobs(doc["knobs"])
    if "server" in stages:
        rows = measure_server()
        best = max(rows, key=lambda r: (r["plans_per_s"], -r["p50_ms"]))
        doc["server"] = {k: best[k] for k in ("fill_poses", "tick_poses", "admit_per_tick")}
        doc["measured_server_batch_64"] = rows
        print("server -> %s" % doc["server"], flush=True)
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
