"""Summaries of rocprofv3 output for the measurement records.

    python -m paper_2306_01301_amd.profsum stats DIR --title T --command C
        kernel statistics (rocprofv3 --kernel-trace --stats, csv) as a
        markdown table
    python -m paper_2306_01301_amd.profsum traffic --fetch DIR --write DIR
        --workload maze_512 --copy-bytes B --command-fetch C --command-write C
        HBM bytes per dispatch from two counter runs (FETCH_SIZE, WRITE_SIZE),
        scaled by what the same counters read for a plain device copy of B
        bytes made first in the profiled program, per sweep kernel kind of
        the benchmark's passes, as JSON

Host code only; it reads the csv files rocprofv3 writes and runs no GPU work.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rows(directory: str, suffix: str):
    files = sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit("no *%s under %s" % (suffix, directory))
    out = []
    for path in files:
        with open(path, newline="") as f:
            out += [{k.strip().lower(): v for k, v in r.items()} for r in csv.DictReader(f)]
    return out


def short_name(name: str) -> str:
    """Kernel name without the argument list and anonymous namespaces."""
    name = name.replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    depth = 0
    for k, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:k].strip()
    return name.strip()


def stats_table(directory: str, title: str, command: str) -> str:
    rows = _rows(directory, "kernel_stats.csv")
    lines = ["# rocprofv3 kernel statistics: %s" % title, "", "Command: `%s`" % command, "",
             "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    rows.sort(key=lambda r: -float(r.get("percentage", 0) or 0))
    for r in rows:
        lines.append("| %s | %s | %.1f | %.1f | %.1f | %.4g |" % (
            short_name(r["name"]), r["calls"], float(r["averagens"]) / 1e3, float(r["minns"]) / 1e3,
            float(r["maxns"]) / 1e3, float(r["percentage"])))
    return "\n".join(lines) + "\n"


def _counter_by_dispatch(directory: str, counter: str):
    """[(dispatch id, kernel name, grid, value)] in dispatch order."""
    vals = defaultdict(float)
    meta = {}
    for r in _rows(directory, "counter_collection.csv"):
        if r.get("counter_name", "").strip() != counter:
            continue
        d = int(r["dispatch_id"])
        vals[d] += float(r["counter_value"])
        meta[d] = (r["kernel_name"], int(r.get("grid_size", 0) or 0))
    return [(d, meta[d][0], meta[d][1], vals[d]) for d in sorted(vals)]


def expected_sweep_kinds(workload: str):
    """Sweep-kernel dispatches of one bench step of `workload`, in order."""
    from . import planner, scenes

    sc = scenes.WORKLOADS[workload]()
    out = []
    for a, b in planner.schedule_passes(sc.schedule, 0, len(sc.schedule) * sc.n_cycles):
        if b >= 0:
            out.append("fused_turn")
        elif a in (planner.SF, planner.SB):
            out += ["straight_y", "straight_x"]  # a straight pass: y-major planes, then x-major planes
        else:
            out.append("turn")
    return out


def traffic(fetch_dir: str, write_dir: str, workload: str, copy_bytes: int, commands) -> dict:
    fetch = _counter_by_dispatch(fetch_dir, "FETCH_SIZE")
    write = _counter_by_dispatch(write_dir, "WRITE_SIZE")
    if [n for _, n, _, _ in fetch] != [n for _, n, _, _ in write]:
        raise SystemExit("the two counter runs dispatched different kernels")

    def calib(rows):
        copies = [v for _, n, _, v in rows if "copy" in n.lower()]
        if not copies:
            raise SystemExit("no copy kernel to calibrate against (run the program with --calibrate-copy)")
        return max(copies) / copy_bytes  # the 1 GiB copy is the largest

    fpb, wpb = calib(fetch), calib(write)
    kernels = {}
    sweeps = []
    for (d, name, grid, fv), (_, _, _, wv) in zip(fetch, write):
        key = "%s grid=%d" % (short_name(name), grid)
        k = kernels.setdefault(key, {"launches": 0, "fetch_bytes": 0.0, "write_bytes": 0.0})
        k["launches"] += 1
        k["fetch_bytes"] += fv / fpb
        k["write_bytes"] += wv / wpb
        if "sweep_kernel" in name or "band_kernel" in name:
            sweeps.append((short_name(name), fv / fpb, wv / wpb))
    for k in kernels.values():
        k["fetch_bytes"] /= k["launches"]
        k["write_bytes"] /= k["launches"]
    want = expected_sweep_kinds(workload)
    if len(sweeps) % len(want):
        raise SystemExit("%d sweep dispatches, not a whole number of %d-launch steps" % (len(sweeps), len(want)))
    per = defaultdict(list)
    names = defaultdict(set)
    for k, (name, fb, wb) in enumerate(sweeps):
        kind = want[k % len(want)]
        per[kind].append((fb, wb))
        names[kind].add(name)
    h = hashlib.sha256()
    for name in ("k_sweep.hip", "nhp_internal.h"):
        with open(os.path.join(ROOT, "paper_2306_01301_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return {
        "command_fetch": commands[0], "command_write": commands[1],
        "calibration": {"copy_bytes": copy_bytes, "fetch_counter_per_byte": fpb, "write_counter_per_byte": wpb},
        "kernels": kernels,
        "sweep_kernels": {kind: sorted(v) for kind, v in names.items()},
        "launches_profiled": {kind: len(v) for kind, v in per.items()},
        "fetch_bytes_per_launch": {kind: sum(f for f, _ in v) / len(v) for kind, v in per.items()},
        "write_bytes_per_launch": {kind: sum(w for _, w in v) / len(v) for kind, v in per.items()},
        "bytes_per_launch": {kind: sum(f + w for f, w in v) / len(v) for kind, v in per.items()},
        "kernel_source_hash": h.hexdigest()[:16],
    }


def gaps(directory: str) -> dict:
    """GPU occupancy of a kernel trace after its last fill kernel (the
    marker the benchmark's batch_64 mode launches): the span from the first
    to the last kernel, the time no kernel runs, and the same inside the
    sweep phase (first to last sweep kernel)."""
    rows = sorted(_rows(directory, "kernel_trace.csv"), key=lambda r: int(r["start_timestamp"]))
    marks = [i for i, r in enumerate(rows) if "fill" in r["kernel_name"].lower()]
    run = rows[marks[-1] + 1:] if marks else rows

    def occupancy(rs):
        iv = sorted((int(r["start_timestamp"]), int(r["end_timestamp"])) for r in rs)
        busy, gap_list = 0, []
        cs, ce = iv[0]
        for s, e in iv[1:]:
            if s > ce:
                busy += ce - cs
                gap_list.append(s - ce)
                cs, ce = s, e
            else:
                ce = max(ce, e)
        busy += ce - cs
        span = iv[-1][1] - iv[0][0]
        gap_list.sort()
        return {"kernels": len(rs), "span_ms": span / 1e6, "busy_ms": busy / 1e6, "idle_frac": 1 - busy / span,
                "gaps": len(gap_list), "largest_gaps_ms": [g / 1e6 for g in gap_list[-5:]]}

    sweeps = [k for k, r in enumerate(run) if "sweep" in r["kernel_name"]]
    inner = run[sweeps[0]:sweeps[-1] + 1] if sweeps else []
    return {"whole_run": occupancy(run), "sweep_phase": occupancy(inner) if inner else None}


def main() -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--workload", default="maze_512")
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    g = sub.add_parser("gaps")
    g.add_argument("dirs", nargs="+")
    a = ap.parse_args()
    if a.cmd == "gaps":
        json.dump({d: gaps(d) for d in a.dirs}, sys.stdout, indent=1)
        sys.stdout.write("\n")
    elif a.cmd == "stats":
        sys.stdout.write(stats_table(a.dir, a.title, a.command))
    else:
        json.dump(traffic(a.fetch, a.write, a.workload, a.copy_bytes, (a.command_fetch, a.command_write)),
                  sys.stdout, indent=1)
        sys.stdout.write("\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
