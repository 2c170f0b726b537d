"""Python binding of libnhp.so (include/nhp.h).

Argument marshalling only: every step of the planner runs in the HIP library.
PyTorch provides the device memory (the plan's workspace is a torch tensor)
and the stream (the current torch stream when the plan is made).  The binding
raises if the library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnhp.so")

INF = 0xFFFFFFFF
HARD = 255
LF, SF, RB, RF, SB, LB = range(6)
NAMES = ("LF", "SF", "RB", "RF", "SB", "LB")
DEFAULT_SCHEDULE = (LF, SF, RB, RF, SB, LB)
MAX_STEPS_DEVICE = 4096

STATUS = {0: "NHP_OK", -1: "NHP_EINVAL", -2: "NHP_ENOMEM", -3: "NHP_EHIP", -4: "NHP_ESTART",
          -5: "NHP_EUNREACH", -6: "NHP_ECAP", -7: "NHP_ESTATE"}
EINVAL, ENOMEM, EHIP, ESTART, EUNREACH, ECAP, ESTATE = -1, -2, -3, -4, -5, -6, -7


class NhpParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_uint32),
        ("ntheta", ctypes.c_uint32),
        ("turn_radius", ctypes.c_double),
        ("ct_q10", ctypes.c_uint32 * 6),
        ("gear_q8", ctypes.c_uint32 * 6),
        ("schedule", ctypes.c_uint8 * 6),
        ("n_schedule", ctypes.c_uint8),
        ("half_cell", ctypes.c_uint8),
        ("reserved", ctypes.c_uint8 * 6),
    ]


class NhpStep(ctypes.Structure):
    _fields_ = [
        ("maneuver", ctypes.c_uint8),
        ("pad", ctypes.c_uint8 * 3),
        ("steps", ctypes.c_uint32),
        ("from_ijt", ctypes.c_uint32 * 3),
        ("to_ijt", ctypes.c_uint32 * 3),
        ("cost_q10", ctypes.c_uint32),
    ]


# name -> (restype, argtypes); the full C ABI of include/nhp.h
_vp, _u32, _i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32
_PU32 = ctypes.POINTER(ctypes.c_uint32)
SIGNATURES = {
    "plan_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(NhpParams)]),
    "plan_create": (ctypes.c_int, [ctypes.POINTER(NhpParams), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "plan_destroy": (ctypes.c_int, [_vp]),
    "plan_set_stream": (ctypes.c_int, [_vp, _vp]),
    "render_cspace": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32]),
    "plan_set_cspace": (ctypes.c_int, [_vp, _vp]),
    "sweep_n_turns": (ctypes.c_int, [_vp, _u32, _u32, _u32, _u32]),
    "sweep_resume": (ctypes.c_int, [_vp, _u32]),
    "sweep_one": (ctypes.c_int, [_vp, _u32]),
    "sweep_pass": (ctypes.c_int, [_vp, _i32, _i32]),
    "sweep_straight_family": (ctypes.c_int, [_vp, _u32, _u32]),
    "sweep_from_set": (ctypes.c_int, [_vp, _vp, _u32, _u32]),
    "soft_cost_image": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32]),
    "extract_path_set": (ctypes.c_int, [_vp, _vp, _vp, _u32, ctypes.POINTER(NhpStep), _u32, _PU32, _PU32, _PU32,
                                        _PU32]),
    "schedule_passes": (ctypes.c_int, [_vp, _u32, ctypes.c_uint64, ctypes.c_uint64, _i32, _vp, _vp, _u32, _PU32]),
    "extract_path": (ctypes.c_int, [_vp, _u32, _u32, _u32, _u32, _u32, _u32, ctypes.POINTER(NhpStep), _u32,
                                    _PU32, _PU32, _PU32, _PU32]),
    "extract_path_noalloc": (ctypes.c_int, [_vp, _u32, _u32, _u32, _u32, _u32, _u32, ctypes.POINTER(NhpStep),
                                            _u32, _PU32, _PU32, _PU32, _PU32]),
    "plan_device_ptrs": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "plan_get_tables": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "plan_last_error": (ctypes.c_char_p, []),
    "nhp_set_section_steps": (ctypes.c_int, [_u32, _u32]),
    "nhp_set_knob": (ctypes.c_int, [_u32, _i32]),
    "nhp_get_knob": (ctypes.c_int32, [_u32]),
    "reach_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(NhpParams), _u32]),
    "reach_create": (ctypes.c_int, [_vp, _u32, _vp, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    "reach_destroy": (ctypes.c_int, [_vp]),
    "reach_render": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32]),
    "reach_set_cspace": (ctypes.c_int, [_vp, _vp]),
    "reach_sweep": (ctypes.c_int, [_vp, _u32, _u32, _u32, _u32]),
    "reach_extract": (ctypes.c_int, [_vp, _u32, _u32, _u32, _u32, ctypes.POINTER(NhpStep), _u32, _PU32, _PU32,
                                     _PU32]),
    "reach_device_ptrs": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "batch_create": (ctypes.c_int, [_u32, _vp, ctypes.POINTER(_vp)]),
    "batch_destroy": (ctypes.c_int, [_vp]),
    "batch_render": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32]),
    "batch_init": (ctypes.c_int, [_vp, _vp, _vp, _u32]),
    "batch_step": (ctypes.c_int, [_vp, _vp, _vp, _u32]),
    "batch_advance": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32]),
    "batch_sweep": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u32]),
    "batch_extract": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp, _vp, ctypes.POINTER(NhpStep), _u32, _vp, _vp,
                                     _vp, _vp, _vp]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Loads libnhp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnhp.so is missing: build it with `python -m paper_2306_01301_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype, fn.argtypes = res, args
        _lib = L
        apply_tuning()
    return _lib


TUNING_PATH = os.path.join(_HERE, "tuning.json")


KNOBS = {"row_wg_per_cu": 0, "xmajor_wg_per_cu": 1, "tile_order": 2, "xmajor_buffers": 3}


def load_tuning(path: str = TUNING_PATH) -> dict:
    import json

    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def apply_tuning_table(table: dict) -> None:
    for length, steps in table.items():
        _lib.nhp_set_section_steps(int(length), int(steps))


def apply_tuning(path: str = TUNING_PATH) -> dict:
    """Hands the measured section sizes and launch knobs (autotune.py) to the library."""
    doc = load_tuning(path)
    table = doc.get("section_steps", {})
    apply_tuning_table(table)
    for name, value in doc.get("knobs", {}).items():
        if name in KNOBS:
            _lib.nhp_set_knob(KNOBS[name], int(value))
    return table


def set_knob(knob: int, value: int) -> None:
    _check(lib().nhp_set_knob(int(knob), int(value)), "nhp_set_knob")


def get_knob(knob: int) -> int:
    return int(lib().nhp_get_knob(int(knob)))


def set_section_steps(curve_len: int, steps: int) -> None:
    _check(lib().nhp_set_section_steps(int(curve_len), int(steps)), "nhp_set_section_steps")


def schedule_passes(schedule: Sequence[int], first_step: int, n_steps: int, pairs: bool = True):
    """The passes (first, second or -1) that the library groups sweeps
    first_step .. first_step + n_steps - 1 of a schedule into."""
    sched = (ctypes.c_uint8 * len(schedule))(*schedule)
    n = ctypes.c_uint32()
    cap = max(1, int(n_steps))
    a, b = (ctypes.c_int8 * cap)(), (ctypes.c_int8 * cap)()
    _check(lib().schedule_passes(sched, len(schedule), int(first_step), int(n_steps), int(bool(pairs)), a, b, cap,
                                 ctypes.byref(n)), "schedule_passes")
    return [(int(a[k]), int(b[k])) for k in range(n.value)]


class NhpError(RuntimeError):
    def __init__(self, rc: int, what: str):
        msg = lib().plan_last_error().decode(errors="replace")
        super().__init__("%s: %s (%s)" % (what, STATUS.get(rc, rc), msg))
        self.rc = rc


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise NhpError(rc, what)


def make_params(nx: int, ntheta: int, turn_radius: float, ct_q10: Sequence[int],
                gear_q8: Sequence[int] = (256,) * 6, schedule: Sequence[int] = DEFAULT_SCHEDULE,
                half_cell: int = 1) -> NhpParams:
    p = NhpParams()
    p.nx, p.ntheta, p.turn_radius = int(nx), int(ntheta), float(turn_radius)
    for k in range(6):
        p.ct_q10[k] = int(ct_q10[k])
        p.gear_q8[k] = int(gear_q8[k])
        p.schedule[k] = int(schedule[k]) if k < len(schedule) else 0
    p.n_schedule = len(schedule)
    p.half_cell = int(half_cell)
    return p


def workspace_bytes(params: NhpParams) -> int:
    return int(lib().plan_workspace_bytes(ctypes.byref(params)))


@dataclass
class Step:
    maneuver: int
    steps: int
    frm: Tuple[int, int, int]
    to: Tuple[int, int, int]
    cost: int


@dataclass
class Path:
    steps: List[Step]
    best: Tuple[int, int, int]
    value: int
    score: int


class NhpStart(ctypes.Structure):
    _fields_ = [("i", ctypes.c_uint32), ("j", ctypes.c_uint32), ("T", ctypes.c_uint32), ("cost_q10", ctypes.c_uint32),
                ("maneuver", ctypes.c_int32)]


MAX_STARTS, MAX_GOALS = 64, 4096


class Planner:
    """One planning problem on one device: owns a workspace tensor and a plan."""

    def __init__(self, nx: int, ntheta: int, turn_radius: float, ct_q10: Sequence[int],
                 gear_q8: Sequence[int] = (256,) * 6, schedule: Sequence[int] = DEFAULT_SCHEDULE,
                 half_cell: int = 1, device: Optional[torch.device] = None,
                 stream: Optional[torch.cuda.Stream] = None, workspace: Optional[torch.Tensor] = None):
        L = lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.params = make_params(nx, ntheta, turn_radius, ct_q10, gear_q8, schedule, half_cell)
        self.nx, self.nt = int(nx), int(ntheta)
        self.schedule = tuple(schedule)
        nbytes = workspace_bytes(self.params)
        if nbytes == 0:
            raise NhpError(EINVAL, "plan_workspace_bytes")
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-workspace.data_ptr()) % 256
        self.ws = workspace[off:off + nbytes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._plan = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.plan_create(ctypes.byref(self.params), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._plan)), "plan_create")
        v, b = ctypes.c_void_p(), ctypes.c_void_p()
        _check(L.plan_device_ptrs(self._plan, ctypes.byref(v), ctypes.byref(b)), "plan_device_ptrs")
        nr = self.nx * self.nx * self.nt
        base = self.ws.data_ptr()
        self._v_off, self._b_off = v.value - base, b.value - base
        self.n_poses = nr

    # ---- views of the plan's device volumes (no copies) ----
    @property
    def value(self) -> torch.Tensor:
        """V as an int32 view [theta, y, x] (reinterpret as uint32 on the host)."""
        nr = self.n_poses
        return self.ws[self._v_off:self._v_off + 4 * nr].view(torch.int32).view(self.nt, self.nx, self.nx)

    @property
    def cspace(self) -> torch.Tensor:
        nr = self.n_poses
        return self.ws[self._b_off:self._b_off + nr].view(self.nt, self.nx, self.nx)

    def value_numpy(self) -> np.ndarray:
        self.stream.synchronize()
        return self.value.cpu().numpy().view(np.uint32)

    def cspace_numpy(self) -> np.ndarray:
        self.stream.synchronize()
        return self.cspace.cpu().numpy()

    # ---- the pipeline ----
    def render(self, image: torch.Tensor, vehicle: Sequence[int]) -> None:
        assert image.dtype == torch.uint8 and image.is_cuda and image.shape == (self.nx, self.nx)
        image = image.contiguous()
        self._image = image  # keep alive until the render has run
        f, r, s = (int(v) for v in vehicle)
        _check(lib().render_cspace(self._plan, ctypes.c_void_p(image.data_ptr()), f, r, s), "render_cspace")

    def set_cspace(self, cspace: torch.Tensor) -> None:
        assert cspace.dtype == torch.uint8 and cspace.is_cuda and cspace.numel() == self.n_poses
        cspace = cspace.contiguous()
        self._cs = cspace
        _check(lib().plan_set_cspace(self._plan, ctypes.c_void_p(cspace.data_ptr())), "plan_set_cspace")

    def sweep(self, start: Sequence[int], n_cycles: int) -> None:
        i, j, t = (int(v) for v in start)
        _check(lib().sweep_n_turns(self._plan, i, j, t, int(n_cycles)), "sweep_n_turns")

    def resume(self, n_cycles: int) -> None:
        _check(lib().sweep_resume(self._plan, int(n_cycles)), "sweep_resume")

    def sweep_one(self, maneuver: int) -> None:
        _check(lib().sweep_one(self._plan, int(maneuver)), "sweep_one")

    def sweep_pass(self, first: int, second: int = -1) -> None:
        """`first` then `second` (-1: none), in one pass when they fuse."""
        _check(lib().sweep_pass(self._plan, int(first), int(second)), "sweep_pass")

    def sweep_straight_family(self, maneuver: int, family: int) -> None:
        """Straight `maneuver` on the planes of one family (1: a row per step, 0: a column per step)."""
        _check(lib().sweep_straight_family(self._plan, int(maneuver), int(family)), "sweep_straight_family")

    def _step_buffer(self, cap: int):
        """A step array of `cap` entries, kept for the next call of the same size."""
        buf = getattr(self, "_steps_buf", None)
        if buf is None or len(buf) != max(1, cap):
            buf = (NhpStep * max(1, cap))()
            self._steps_buf = buf
        return buf

    def extract(self, goal: Sequence[int], radius: int = 0, w_xy: int = 1024, w_t: int = 1024,
                cap: int = MAX_STEPS_DEVICE) -> Path:
        steps = self._step_buffer(cap)
        n, best, val, score = ctypes.c_uint32(), (ctypes.c_uint32 * 3)(), ctypes.c_uint32(), ctypes.c_uint32()
        gi, gj, gt = (int(v) for v in goal)
        rc = lib().extract_path(self._plan, gi, gj, gt, int(radius), int(w_xy), int(w_t), steps, int(cap),
                                ctypes.byref(n), best, ctypes.byref(val), ctypes.byref(score))
        _check(rc, "extract_path")
        out = [Step(int(s.maneuver), int(s.steps), tuple(int(v) for v in s.from_ijt),
                    tuple(int(v) for v in s.to_ijt), int(s.cost_q10)) for s in steps[: n.value]]
        return Path(out, tuple(int(v) for v in best), int(val.value), int(score.value))

    def extract_noalloc(self, goal: Sequence[int], radius: int = 0, w_xy: int = 1024, w_t: int = 1024,
                        steps=None) -> Path:
        """extract_path_noalloc: as extract, with the library's fixed extract
        area.  `steps`: a caller-made NhpStep array (default: the planner's
        cached one of MAX_STEPS_DEVICE entries)."""
        if steps is None:
            steps = self._step_buffer(MAX_STEPS_DEVICE)
        n, best, val, score = ctypes.c_uint32(), (ctypes.c_uint32 * 3)(), ctypes.c_uint32(), ctypes.c_uint32()
        gi, gj, gt = (int(v) for v in goal)
        rc = lib().extract_path_noalloc(self._plan, gi, gj, gt, int(radius), int(w_xy), int(w_t), steps, len(steps),
                                        ctypes.byref(n), best, ctypes.byref(val), ctypes.byref(score))
        _check(rc, "extract_path_noalloc")
        out = [Step(int(s.maneuver), int(s.steps), tuple(int(v) for v in s.from_ijt),
                    tuple(int(v) for v in s.to_ijt), int(s.cost_q10)) for s in steps[: n.value]]
        return Path(out, tuple(int(v) for v in best), int(val.value), int(score.value))

    def soft_costs(self, image: torch.Tensor, table) -> torch.Tensor:
        """Codes from the squared distance to the nearest hard pixel (an nx x
        nx device image in, a new device image out)."""
        assert image.dtype == torch.uint8 and image.is_cuda and image.shape == (self.nx, self.nx)
        image = image.contiguous()
        out = torch.empty_like(image)
        tab = np.ascontiguousarray(np.asarray(table, np.uint8))
        _check(lib().soft_cost_image(self._plan, ctypes.c_void_p(image.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                     tab.ctypes.data, len(tab)), "soft_cost_image")
        return out

    def sweep_from_set(self, starts, n_cycles: int) -> None:
        """starts: (i, j, T, cost_q10) at rest or (i, j, T, cost_q10, maneuver)
        with that maneuver in progress."""
        arr = (NhpStart * len(starts))()
        for k, st in enumerate(starts):
            arr[k] = NhpStart(int(st[0]), int(st[1]), int(st[2]), int(st[3]), int(st[4]) if len(st) > 4 else -1)
        _check(lib().sweep_from_set(self._plan, arr, len(starts), int(n_cycles)), "sweep_from_set")

    def extract_set(self, goals, penalty, cap: int = MAX_STEPS_DEVICE):
        """Goal set with penalties; returns (Path, index of the chosen goal)."""
        g = np.ascontiguousarray(np.asarray(goals, np.uint32).reshape(-1))
        pen = np.ascontiguousarray(np.asarray(penalty, np.uint32))
        steps = self._step_buffer(cap)
        n, k, val, score = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        rc = lib().extract_path_set(self._plan, g.ctypes.data, pen.ctypes.data, len(pen), steps, int(cap),
                                    ctypes.byref(n), ctypes.byref(k), ctypes.byref(val), ctypes.byref(score))
        _check(rc, "extract_path_set")
        out = [Step(int(s.maneuver), int(s.steps), tuple(int(v) for v in s.from_ijt),
                    tuple(int(v) for v in s.to_ijt), int(s.cost_q10)) for s in steps[: n.value]]
        best = tuple(int(v) for v in g[3 * k.value: 3 * k.value + 3])
        return Path(out, best, int(val.value), int(score.value)), int(k.value)

    def tables(self) -> dict:
        L, N = self.nt, self.nx
        out = dict(beta=np.zeros(L, np.int32), psi=np.zeros(L, np.int32), I=np.zeros(L, np.int32),
                   J=np.zeros(L, np.int32), Bsk=np.zeros((L, N), np.int32), Lq=np.zeros((6, L), np.uint32))
        _check(lib().plan_get_tables(self._plan, *[ctypes.c_void_p(out[k].ctypes.data) for k in
                                                   ("beta", "psi", "I", "J", "Bsk", "Lq")]), "plan_get_tables")
        return out

    def set_stream(self, stream: torch.cuda.Stream) -> None:
        self.stream = stream
        _check(lib().plan_set_stream(self._plan, ctypes.c_void_p(stream.cuda_stream)), "plan_set_stream")

    def close(self) -> None:
        if getattr(self, "_plan", None) is not None and self._plan.value:
            lib().plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def planner_for(scene, **kw) -> Planner:
    """A Planner with a scene's parameters (see scenes.Scene)."""
    return Planner(scene.nx, scene.nt, scene.R, scene.ct, scene.gear, scene.schedule, scene.half_cell, **kw)


def plan_scene(scene, radius: Optional[int] = None, device=None) -> Tuple[Planner, Path]:
    """Render, sweep and extract one scene on the GPU."""
    p = planner_for(scene, device=device)
    img = torch.from_numpy(np.ascontiguousarray(scene.image)).to(p.device)
    p.render(img, scene.vehicle)
    p.sweep(scene.start, scene.n_cycles)
    path = p.extract(scene.goal, scene.goal_radius if radius is None else radius, scene.w_xy, scene.w_t)
    return p, path


def _u32array(values) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(values, dtype=np.uint32).reshape(-1))


class Batch:
    """Batched launches over many plans (include/nhp.h, batch_*): one launch
    per pass covers the current work of every listed plan."""

    def __init__(self, capacity: int, stream: Optional[torch.cuda.Stream] = None):
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._b = ctypes.c_void_p()
        _check(lib().batch_create(int(capacity), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._b)),
               "batch_create")
        self.capacity = int(capacity)

    @staticmethod
    def _handles(planners):
        arr = (ctypes.c_void_p * max(1, len(planners)))()
        for k, p in enumerate(planners):
            arr[k] = p._plan.value
        return arr

    def render(self, planners, images, vehicles) -> None:
        imgs = [im.contiguous() for im in images]
        self._keep = imgs
        ptrs = (ctypes.c_void_p * max(1, len(imgs)))(*[im.data_ptr() for im in imgs])
        boxes = np.ascontiguousarray(np.asarray(vehicles, dtype=np.int32).reshape(-1))
        _check(lib().batch_render(self._b, self._handles(planners), ptrs, boxes.ctypes.data, len(planners)),
               "batch_render")

    def init(self, planners, starts) -> None:
        s = _u32array(starts)
        _check(lib().batch_init(self._b, self._handles(planners), s.ctypes.data, len(planners)), "batch_init")

    def step(self, planners, steps) -> None:
        s = _u32array(steps)
        _check(lib().batch_step(self._b, self._handles(planners), s.ctypes.data, len(planners)), "batch_step")

    def advance(self, planners, steps, counts) -> None:
        """Plan k runs sweeps steps[k] .. steps[k] + counts[k] - 1 (fusing
        consecutive turns on shared circles)."""
        s, c = _u32array(steps), _u32array(counts)
        _check(lib().batch_advance(self._b, self._handles(planners), s.ctypes.data, c.ctypes.data, len(planners)),
               "batch_advance")

    def sweep(self, planners, starts, n_cycles) -> None:
        s, n = _u32array(starts), _u32array(n_cycles)
        _check(lib().batch_sweep(self._b, self._handles(planners), s.ctypes.data, n.ctypes.data, len(planners)),
               "batch_sweep")

    def extract(self, planners, goals, radius, w_xy, w_t, cap: int = 512):
        """Returns a list with a Path or an NhpError status code per plan."""
        n = len(planners)
        g, r, wx, wt = _u32array(goals), _u32array(radius), _u32array(w_xy), _u32array(w_t)
        steps = (NhpStep * max(1, n * cap))()
        n_steps = np.zeros(n, np.uint32)
        status = np.zeros(n, np.int32)
        best = np.zeros(3 * n, np.uint32)
        val = np.zeros(n, np.uint32)
        score = np.zeros(n, np.uint32)
        _check(lib().batch_extract(self._b, self._handles(planners), n, g.ctypes.data, r.ctypes.data,
                                   wx.ctypes.data, wt.ctypes.data, steps, int(cap), n_steps.ctypes.data,
                                   status.ctypes.data, best.ctypes.data, val.ctypes.data, score.ctypes.data),
               "batch_extract")
        out = []
        for k in range(n):
            if status[k] != 0:
                out.append(int(status[k]))
                continue
            ss = steps[k * cap:k * cap + int(n_steps[k])]
            out.append(Path([Step(int(s.maneuver), int(s.steps), tuple(int(v) for v in s.from_ijt),
                                  tuple(int(v) for v in s.to_ijt), int(s.cost_q10)) for s in ss],
                            tuple(int(v) for v in best[3 * k:3 * k + 3]), int(val[k]), int(score[k])))
        return out

    def close(self) -> None:
        if getattr(self, "_b", None) is not None and self._b.value:
            lib().batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class ReachPath:
    steps: List[Step]
    best: Tuple[int, int, int]
    level: int  # maneuvers used


class Reach:
    """Maneuver-count reachability (App. C) on a planner's tables and
    stream: obstacle bits and level bit volumes in a workspace tensor."""

    def __init__(self, planner: Planner, max_cycles: int, workspace: Optional[torch.Tensor] = None):
        L = lib()
        self.planner = planner
        self.max_cycles = int(max_cycles)
        nbytes = int(L.reach_workspace_bytes(ctypes.byref(planner.params), self.max_cycles))
        if nbytes == 0:
            raise NhpError(EINVAL, "reach_workspace_bytes")
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=planner.device)
        off = (-workspace.data_ptr()) % 256
        self.ws = workspace[off:off + nbytes]
        self._r = ctypes.c_void_p()
        with torch.cuda.device(planner.device):
            _check(L.reach_create(planner._plan, self.max_cycles, ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                  ctypes.byref(self._r)), "reach_create")
        h, v = ctypes.c_void_p(), ctypes.c_void_p()
        _check(L.reach_device_ptrs(self._r, ctypes.byref(h), ctypes.byref(v)), "reach_device_ptrs")
        base = self.ws.data_ptr()
        self._h_off, self._l_off = h.value - base, v.value - base
        self.words = planner.n_poses // 32

    def hard_words(self) -> torch.Tensor:
        return self.ws[self._h_off:self._h_off + 4 * self.words].view(torch.int32)

    def level_words(self, m: int) -> torch.Tensor:
        o = self._l_off + 4 * self.words * int(m)
        return self.ws[o:o + 4 * self.words].view(torch.int32)

    def render(self, image: torch.Tensor, vehicle: Sequence[int]) -> None:
        assert image.dtype == torch.uint8 and image.is_cuda and image.shape == (self.planner.nx, self.planner.nx)
        image = image.contiguous()
        self._image = image
        f, r, s = (int(v) for v in vehicle)
        _check(lib().reach_render(self._r, ctypes.c_void_p(image.data_ptr()), f, r, s), "reach_render")

    def set_cspace(self, codes: torch.Tensor) -> None:
        assert codes.dtype == torch.uint8 and codes.is_cuda and codes.numel() == self.planner.n_poses
        codes = codes.contiguous()
        self._codes = codes
        _check(lib().reach_set_cspace(self._r, ctypes.c_void_p(codes.data_ptr())), "reach_set_cspace")

    def sweep(self, start: Sequence[int], n_cycles: int) -> None:
        i, j, t = (int(v) for v in start)
        _check(lib().reach_sweep(self._r, i, j, t, int(n_cycles)), "reach_sweep")

    def extract(self, goal: Sequence[int], radius: int = 0, cap: int = 256) -> ReachPath:
        steps = (NhpStep * max(1, cap))()
        n, best, lv = ctypes.c_uint32(), (ctypes.c_uint32 * 3)(), ctypes.c_uint32()
        gi, gj, gt = (int(v) for v in goal)
        _check(lib().reach_extract(self._r, gi, gj, gt, int(radius), steps, int(cap), ctypes.byref(n), best,
                                   ctypes.byref(lv)), "reach_extract")
        out = [Step(int(s.maneuver), int(s.steps), tuple(int(v) for v in s.from_ijt),
                    tuple(int(v) for v in s.to_ijt), int(s.cost_q10)) for s in steps[: n.value]]
        return ReachPath(out, tuple(int(v) for v in best), int(lv.value))

    def close(self) -> None:
        if getattr(self, "_r", None) is not None and self._r.value:
            self.planner.stream.synchronize()
            lib().reach_destroy(self._r)
            self._r = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bits_to_levels(words: Sequence[np.ndarray], shape) -> np.ndarray:
    """Per-pose level (smallest m whose volume has the pose's bit clear, 255
    if none) from level volumes given as uint32 word arrays."""
    level = np.full(int(np.prod(shape)), 255, np.uint8)
    for m, w in enumerate(words):
        bits = np.unpackbits(np.asarray(w, np.uint32).view(np.uint8), bitorder="little").astype(bool)
        level[(~bits) & (level == 255)] = m
    return level.reshape(shape)
