"""CPU oracle of the kernel-style N-turn planner (arXiv 2306.01301).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2306_01301_amd``) never imports it, and it imports nothing from the
product.

This module is argument marshalling around ``nhp_oracle.c`` (ctypes + numpy);
the arithmetic lives in the C file, which cites the paper step by step.

Volumes are numpy arrays of shape (N_theta, N, N), index [T, j, i].
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nhp_oracle.c")
_LIB = os.path.join(_HERE, "libnhp_oracle.so")

INF = 0xFFFFFFFF
HARD = 255
LF, SF, RB, RF, SB, LB = range(6)
NAMES = ["LF", "SF", "RB", "RF", "SB", "LB"]
DEFAULT_SCHEDULE = [LF, SF, RB, RF, SB, LB]

OK, EINVAL, ENOMEM, ESTART, EUNREACH, ECAP = 0, -1, -2, -4, -5, -6


_LIB_NATIVE = os.path.join(_HERE, "libnhp_oracle_native.so")
_active = _LIB


def build(force: bool = False, native: bool = False) -> str:
    """Compiles the oracle shared library in place (gcc, OpenMP).

    native: builds a second copy with -O3 -march=native for the host it runs
    on (always rebuilt, since the host may differ from the one that built
    the first) and makes the module use it from then on; the timing
    baseline runs on it.  Floating-point contraction stays off, so the
    tables come out the same either way."""
    global _active, _lib
    target = _LIB_NATIVE if native else _LIB
    opt = ["-O3", "-march=native", "-ffp-contract=off"] if native else ["-O2"]
    if force or native or not os.path.exists(target) or os.path.getmtime(target) < os.path.getmtime(_SRC):
        tmp = target + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc"] + opt + ["-std=c99", "-Wall", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, target)
    if native and _active != target:
        _active, _lib = target, None
    return target


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32),
        ("nt", ctypes.c_int32),
        ("R", ctypes.c_double),
        ("half_cell", ctypes.c_int32),
        ("nsched", ctypes.c_int32),
        ("sched", ctypes.c_int32 * 6),
        ("ct", ctypes.c_uint32 * 6),
        ("gear", ctypes.c_uint32 * 6),
    ]


class _Step(ctypes.Structure):
    _fields_ = [
        ("maneuver", ctypes.c_uint8),
        ("pad", ctypes.c_uint8 * 3),
        ("steps", ctypes.c_uint32),
        ("from_", ctypes.c_uint32 * 3),
        ("to", ctypes.c_uint32 * 3),
        ("cost", ctypes.c_uint32),
    ]


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_active):
            build()
        lib = ctypes.CDLL(_active)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        i32 = ctypes.c_int32
        u32 = ctypes.c_uint32
        lib.or_tables_export.argtypes = [P(_Problem), vp, vp, vp, vp, vp, vp]
        lib.or_render_taps.argtypes = [P(_Problem), i32, i32, i32, i32, vp, vp, vp, vp]
        lib.or_render.argtypes = [P(_Problem), vp, i32, i32, i32, vp]
        lib.or_init.argtypes = [P(_Problem), vp, vp, i32, i32, i32]
        lib.or_sweep.argtypes = [P(_Problem), i32, vp, vp]
        lib.or_cycles.argtypes = [P(_Problem), vp, vp, i32]
        lib.or_goal_search.argtypes = [P(_Problem), vp, vp, i32, i32, i32, i32, u32, u32, vp, vp]
        lib.or_backtrack.argtypes = [P(_Problem), vp, vp, i32, i32, i32, vp, vp, i32, vp]
        lib.or_set_threads.argtypes = [i32]
        lib.or_init_set.argtypes = [P(_Problem), vp, vp, vp, i32]
        lib.or_soft_costs.argtypes = [vp, i32, vp, i32, vp]
        lib.or_goal_set.argtypes = [P(_Problem), vp, vp, vp, vp, i32, vp, vp]
        lib.or_backtrack_set.argtypes = [P(_Problem), vp, vp, vp, i32, vp, vp, i32, vp]
        lib.or_reach.argtypes = [P(_Problem), vp, i32, i32, i32, i32, vp]
        lib.or_reach_goal.argtypes = [P(_Problem), vp, i32, i32, i32, i32, vp, vp]
        lib.or_reach_backtrack.argtypes = [P(_Problem), vp, vp, vp, vp, i32, vp]
        for name in ("or_tables_export", "or_render_taps", "or_render", "or_init", "or_sweep",
                     "or_cycles", "or_goal_search", "or_backtrack", "or_set_threads", "or_reach",
                     "or_init_set", "or_goal_set", "or_backtrack_set", "or_soft_costs",
                     "or_reach_goal", "or_reach_backtrack"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__("%s failed with status %d" % (what, rc))
        self.rc = rc


def _check(rc: int, what: str) -> None:
    if rc != OK:
        raise OracleError(rc, what)


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


@dataclass
class Problem:
    """The planner's parameters (graph of Sec. V, costs of Sec. VI/XIV)."""

    nx: int
    nt: int
    R: float
    half_cell: int = 1
    schedule: Sequence[int] = field(default_factory=lambda: list(DEFAULT_SCHEDULE))
    ct: Sequence[int] = field(default_factory=lambda: [0] * 6)
    gear: Sequence[int] = field(default_factory=lambda: [256] * 6)

    def c(self) -> _Problem:
        p = _Problem()
        p.nx, p.nt, p.R, p.half_cell = int(self.nx), int(self.nt), float(self.R), int(self.half_cell)
        p.nsched = len(self.schedule)
        for k in range(6):
            p.sched[k] = int(self.schedule[k]) if k < len(self.schedule) else 0
            p.ct[k] = int(self.ct[k])
            p.gear[k] = int(self.gear[k])
        return p

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nt, self.nx, self.nx)


def set_threads(n: int) -> int:
    """Sets the OpenMP thread count of the oracle; returns the count in effect."""
    return int(_L().or_set_threads(int(n)))


def tables(prob: Problem) -> dict:
    L, N = prob.nt, prob.nx
    out = dict(
        beta=np.zeros(L, np.int32), psi=np.zeros(L, np.int32), I=np.zeros(L, np.int32),
        J=np.zeros(L, np.int32), Bsk=np.zeros((L, N), np.int32), Lq=np.zeros((6, L), np.uint32),
    )
    p = prob.c()
    _check(_L().or_tables_export(ctypes.byref(p), *[_ptr(out[k]) for k in
                                                     ("beta", "psi", "I", "J", "Bsk", "Lq")]),
           "or_tables_export")
    return out


def render_taps(prob: Problem, T: int, f: int, r: int, s: int):
    sdx = np.zeros(2 * s + 1, np.int32)
    sdy = np.zeros(2 * s + 1, np.int32)
    ldx = np.zeros(f + r + 1, np.int32)
    ldy = np.zeros(f + r + 1, np.int32)
    p = prob.c()
    _check(_L().or_render_taps(ctypes.byref(p), T, f, r, s, _ptr(sdx), _ptr(sdy), _ptr(ldx), _ptr(ldy)),
           "or_render_taps")
    return sdx, sdy, ldx, ldy


def render(prob: Problem, image: np.ndarray, f: int, r: int, s: int) -> np.ndarray:
    image = np.ascontiguousarray(image, dtype=np.uint8)
    assert image.shape == (prob.nx, prob.nx)
    B = np.zeros(prob.shape, np.uint8)
    p = prob.c()
    _check(_L().or_render(ctypes.byref(p), _ptr(image), f, r, s, _ptr(B)), "or_render")
    return B


def init(prob: Problem, B: np.ndarray, start: Sequence[int]) -> np.ndarray:
    V = np.zeros(prob.shape, np.uint32)
    p = prob.c()
    _check(_L().or_init(ctypes.byref(p), _ptr(B), _ptr(V), *[int(v) for v in start]), "or_init")
    return V


def sweep(prob: Problem, mu: int, B: np.ndarray, V: np.ndarray) -> None:
    """One maneuver kernel applied to V in place."""
    assert V.dtype == np.uint32 and B.dtype == np.uint8
    p = prob.c()
    _check(_L().or_sweep(ctypes.byref(p), int(mu), _ptr(B), _ptr(V)), "or_sweep")


def cycles(prob: Problem, B: np.ndarray, V: np.ndarray, n_cycles: int) -> None:
    assert V.dtype == np.uint32 and B.dtype == np.uint8
    p = prob.c()
    _check(_L().or_cycles(ctypes.byref(p), _ptr(B), _ptr(V), int(n_cycles)), "or_cycles")


def goal_search(prob: Problem, B, V, goal, d: int, w_xy: int, w_t: int):
    best = np.zeros(3, np.int32)
    score = np.zeros(1, np.uint32)
    p = prob.c()
    _check(_L().or_goal_search(ctypes.byref(p), _ptr(B), _ptr(V), *[int(v) for v in goal], int(d),
                               int(w_xy), int(w_t), _ptr(best), _ptr(score)), "or_goal_search")
    return tuple(int(v) for v in best), int(score[0])


@dataclass
class Step:
    maneuver: int
    steps: int
    frm: Tuple[int, int, int]
    to: Tuple[int, int, int]
    cost: int


def backtrack(prob: Problem, B, V, start, best, cap: int = 4096) -> List[Step]:
    steps = (_Step * max(cap, 1))()
    n = ctypes.c_int32(0)
    g = np.array(best, np.int32)
    p = prob.c()
    _check(_L().or_backtrack(ctypes.byref(p), _ptr(B), _ptr(V), *[int(v) for v in start], _ptr(g),
                             ctypes.addressof(steps), int(cap), ctypes.addressof(n)), "or_backtrack")
    return [Step(int(s.maneuver), int(s.steps), tuple(int(v) for v in s.from_), tuple(int(v) for v in s.to),
                 int(s.cost)) for s in steps[: n.value]]


def plan(prob: Problem, image, vehicle, start, goal, n_cycles, d=0, w_xy=0, w_t=0):
    """Render, init, N cycles, goal search, back-track.  Returns a dict."""
    f, r, s = vehicle
    B = render(prob, image, f, r, s)
    V = init(prob, B, start)
    cycles(prob, B, V, n_cycles)
    best, score = goal_search(prob, B, V, goal, d, w_xy, w_t)
    steps = backtrack(prob, B, V, start, best)
    return dict(B=B, V=V, best=best, score=score, steps=steps)


# ---------------------------------------------------------------- App. C

UNREACHED = 255


def reach(prob: Problem, B: np.ndarray, start, n_cycles: int) -> np.ndarray:
    """Maneuver-count reachability (hard obstacles only): per vertex the
    smallest m <= n_cycles with the vertex reachable in m maneuvers, else 255."""
    assert B.dtype == np.uint8
    level = np.empty(B.shape, np.uint8)
    p = prob.c()
    _check(_L().or_reach(ctypes.byref(p), _ptr(B), *[int(v) for v in start], int(n_cycles), _ptr(level)),
           "or_reach")
    return level


def reach_goal(prob: Problem, level: np.ndarray, goal, d: int):
    best = np.zeros(3, np.int32)
    lv = np.zeros(1, np.int32)
    p = prob.c()
    _check(_L().or_reach_goal(ctypes.byref(p), _ptr(level), *[int(v) for v in goal], int(d), _ptr(best), _ptr(lv)),
           "or_reach_goal")
    return tuple(int(v) for v in best), int(lv[0])


def reach_backtrack(prob: Problem, B, level, best, cap: int = 1024) -> List[Step]:
    steps = (_Step * max(cap, 1))()
    n = ctypes.c_int32(0)
    g = np.array(best, np.int32)
    p = prob.c()
    _check(_L().or_reach_backtrack(ctypes.byref(p), _ptr(B), _ptr(level), _ptr(g), ctypes.addressof(steps),
                                   int(cap), ctypes.addressof(n)), "or_reach_backtrack")
    return [Step(int(s.maneuver), int(s.steps), tuple(int(v) for v in s.from_), tuple(int(v) for v in s.to),
                 int(s.cost)) for s in steps[: n.value]]


# ---------------------------------------------------------------- start and goal sets

class _Start(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int32), ("j", ctypes.c_int32), ("T", ctypes.c_int32), ("cost", ctypes.c_uint32),
                ("maneuver", ctypes.c_int32)]


def _starts(starts):
    """starts: sequence of (i, j, T, cost) or (i, j, T, cost, maneuver)."""
    arr = (_Start * len(starts))()
    for k, s in enumerate(starts):
        mu = s[4] if len(s) > 4 else -1
        arr[k] = _Start(int(s[0]), int(s[1]), int(s[2]), int(s[3]), int(mu))
    return arr


def init_set(prob: Problem, B: np.ndarray, starts) -> np.ndarray:
    V = np.empty(B.shape, np.uint32)
    p = prob.c()
    arr = _starts(starts)
    _check(_L().or_init_set(ctypes.byref(p), _ptr(B), _ptr(V), ctypes.addressof(arr), len(starts)), "or_init_set")
    return V


def goal_set(prob: Problem, B, V, goals, penalty):
    g = np.ascontiguousarray(np.asarray(goals, np.int32).reshape(-1))
    pen = np.ascontiguousarray(np.asarray(penalty, np.uint32))
    k = np.zeros(1, np.int32)
    sc = np.zeros(1, np.uint32)
    p = prob.c()
    _check(_L().or_goal_set(ctypes.byref(p), _ptr(B), _ptr(V), _ptr(g), _ptr(pen), len(pen), _ptr(k), _ptr(sc)),
           "or_goal_set")
    return int(k[0]), int(sc[0])


def backtrack_set(prob: Problem, B, V, starts, best, cap: int = 4096) -> List[Step]:
    steps = (_Step * max(cap, 1))()
    n = ctypes.c_int32(0)
    g = np.array(best, np.int32)
    arr = _starts(starts)
    p = prob.c()
    _check(_L().or_backtrack_set(ctypes.byref(p), _ptr(B), _ptr(V), ctypes.addressof(arr), len(starts), _ptr(g),
                                 ctypes.addressof(steps), int(cap), ctypes.addressof(n)), "or_backtrack_set")
    return [Step(int(s.maneuver), int(s.steps), tuple(int(v) for v in s.from_), tuple(int(v) for v in s.to),
                 int(s.cost)) for s in steps[: n.value]]


def soft_costs(image: np.ndarray, table) -> np.ndarray:
    """Codes from the squared distance to the nearest hard pixel (Sec. VI)."""
    img = np.ascontiguousarray(image, np.uint8)
    n = img.shape[0]
    assert img.shape == (n, n)
    tab = np.ascontiguousarray(np.asarray(table, np.uint8))
    out = np.empty_like(img)
    _check(_L().or_soft_costs(_ptr(img), n, _ptr(tab), len(tab), _ptr(out)), "or_soft_costs")
    return out
