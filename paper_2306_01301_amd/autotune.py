"""Autotuner for the sweep kernels' section size.

A sweep workgroup owns 64 curves and splits each curve into sections of P
steps held by one wave each.  Every valid P (8, 16, 32 or 64 with at most 16
sections) gives identical results; the speed differs with the curve length,
the grid and the chip.  This measures each candidate with HIP events on
free-space volumes and writes the fastest per curve length to tuning.json,
which the binding hands to the library (nhp_set_section_steps) when it loads.

    python -m paper_2306_01301_amd.autotune [--lengths 64,128,256,384,512,1024]
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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--lengths", default="64,72,128,200,256,384,512,1024")
    ap.add_argument("--out", default=P.TUNING_PATH)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    P.lib()
    table, measured = {}, {}
    for length in [int(x) for x in args.lengths.split(",") if x]:
        if length % 8 or length < 16:
            continue
        ms = measure(length)
        best = min(ms, key=ms.get)
        table[str(length)] = best
        measured[str(length)] = {str(k): round(v, 4) for k, v in ms.items()}
        print("length %4d: %s -> %d" % (length, measured[str(length)], best), flush=True)
    doc = {"device": torch.cuda.get_device_name(0), "section_steps": table,
           "measured_ms_turn_plus_straight": measured}
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
