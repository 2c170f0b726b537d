"""Seeded synthetic planning inputs.

This module only draws inputs: obstacle images (uint8 cost codes, 255 = hard),
vehicle boxes, start/goal poses and planner parameters.  It holds none of the
planner's arithmetic (no tables, rendering, sweeps or back-tracking), so both
the HIP path and the CPU oracle may take their inputs from it.

The paper's own scenes (parking, free space, mazes; Sec. XVI) exist only as
figures, so these generators stand in for them with the same shapes and sizes.
Every generator is deterministic in its seed (numpy PCG64).

Cost codes: 0..254 soft (slowness grows with the code), 255 hard.
Coordinates: image[j, i] is row j (y), column i (x); poses are (i, j, T).
Costs are in 1/1024 cell (Q10); gear factors in 1/256 (Q8).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

HARD = 255
LF, SF, RB, RF, SB, LB = range(6)
DEFAULT_SCHEDULE = (LF, SF, RB, RF, SB, LB)
FORWARD_SCHEDULE = (LF, SF, RF)
Q10 = 1024


@dataclass
class Scene:
    name: str
    nx: int
    nt: int
    R: float
    image: np.ndarray
    vehicle: Tuple[int, int, int]  # (front, rear, half width) in cells from the rear axle
    start: Tuple[int, int, int]
    goal: Tuple[int, int, int]
    n_cycles: int
    ct: Tuple[int, ...] = (0,) * 6
    gear: Tuple[int, ...] = (256,) * 6
    schedule: Tuple[int, ...] = DEFAULT_SCHEDULE
    half_cell: int = 1
    goal_radius: int = 0
    w_xy: int = Q10
    w_t: int = Q10
    seed: int = 0

    @property
    def n_poses(self) -> int:
        return self.nx * self.nx * self.nt

    def with_(self, **kw) -> "Scene":
        return replace(self, **kw)


def vehicle_box(length: int, width: int) -> Tuple[int, int, int]:
    """Box extents from the rear axle: about a fifth of the length behind it
    (the paper's example car is 3.65 m forward and 0.85 m back of 4.5 m)."""
    rear = int(round(0.19 * (length - 1)))
    return (length - 1 - rear, rear, width // 2)


def uniform_ct(cells: float) -> Tuple[int, ...]:
    return (int(round(cells * Q10)),) * 6


def reverse_gear(factor_q8: int) -> Tuple[int, ...]:
    g = [256] * 6
    for mu in (RB, SB, LB):
        g[mu] = factor_q8
    return tuple(g)


# ---------------------------------------------------------------------------
# pose sampling (conservative: the whole disk that can hold the footprint is
# free in the image, and the disk keeps away from the one-cell walls)
# ---------------------------------------------------------------------------

def footprint_radius(vehicle: Sequence[int]) -> float:
    f, r, s = vehicle
    return float(np.hypot(max(f, r), s)) + 1.0


def pose_is_clear(image: np.ndarray, i: int, j: int, vehicle: Sequence[int]) -> bool:
    n = image.shape[0]
    rad = footprint_radius(vehicle)
    lo, hi = int(np.floor(rad)) + 1, n - int(np.ceil(rad)) - 1
    if not (lo <= i < hi and lo <= j < hi):
        return False
    k = int(np.ceil(rad))
    ys, xs = np.mgrid[-k:k + 1, -k:k + 1]
    mask = xs * xs + ys * ys <= rad * rad
    patch = image[j - k:j + k + 1, i - k:i + k + 1]
    return bool(np.all(patch[mask] != HARD))


def sample_pose(rng: np.random.Generator, image: np.ndarray, nt: int, vehicle, tries: int = 100000):
    n = image.shape[0]
    for _ in range(tries):
        i, j = int(rng.integers(0, n)), int(rng.integers(0, n))
        if pose_is_clear(image, i, j, vehicle):
            return (i, j, int(rng.integers(0, nt)))
    raise RuntimeError("no clear pose found")


# ---------------------------------------------------------------------------
# obstacle images
# ---------------------------------------------------------------------------

def rect_clutter(rng, n: int, n_rect: int, side_lo: int, side_hi: int) -> np.ndarray:
    img = np.zeros((n, n), np.uint8)
    for _ in range(n_rect):
        w, h = int(rng.integers(side_lo, side_hi + 1)), int(rng.integers(side_lo, side_hi + 1))
        x, y = int(rng.integers(0, n - w + 1)), int(rng.integers(0, n - h + 1))
        img[y:y + h, x:x + w] = HARD
    return img


def mixed_clutter(rng, n: int, occupancy: float) -> np.ndarray:
    """Rectangles (sides 2..16) and disks (radius 2..10) until the hard
    fraction reaches `occupancy`."""
    img = np.zeros((n, n), np.uint8)
    target = occupancy * n * n
    filled = 0
    while filled < target:
        if rng.random() < 0.5:
            w, h = int(rng.integers(2, 17)), int(rng.integers(2, 17))
            x, y = int(rng.integers(0, n - w + 1)), int(rng.integers(0, n - h + 1))
            patch = img[y:y + h, x:x + w]
            filled += int(np.count_nonzero(patch != HARD))
            patch[:] = HARD
        else:
            rad = int(rng.integers(2, 11))
            cx, cy = int(rng.integers(0, n)), int(rng.integers(0, n))
            y0, y1, x0, x1 = max(0, cy - rad), min(n, cy + rad + 1), max(0, cx - rad), min(n, cx + rad + 1)
            yy, xx = np.mgrid[y0:y1, x0:x1]
            disk = (xx - cx) ** 2 + (yy - cy) ** 2 <= rad * rad
            patch = img[y0:y1, x0:x1]
            filled += int(np.count_nonzero(disk & (patch != HARD)))
            patch[disk] = HARD
    return img


def maze(rng, n_cells: int, pitch: int, wall: int) -> np.ndarray:
    """Recursive-backtracker maze: n_cells x n_cells maze cells of `pitch`
    pixels, walls `wall` pixels thick on the low side of every cell."""
    n = n_cells * pitch
    img = np.zeros((n, n), np.uint8)
    for k in range(n_cells):
        img[k * pitch:k * pitch + wall, :] = HARD
        img[:, k * pitch:k * pitch + wall] = HARD
    seen = np.zeros((n_cells, n_cells), bool)
    stack = [(0, 0)]
    seen[0, 0] = True
    while stack:
        a, b = stack[-1]
        nbrs = [(a + da, b + db) for da, db in ((1, 0), (-1, 0), (0, 1), (0, -1))
                if 0 <= a + da < n_cells and 0 <= b + db < n_cells and not seen[a + da, b + db]]
        if not nbrs:
            stack.pop()
            continue
        a2, b2 = nbrs[int(rng.permutation(len(nbrs))[0])]
        seen[a2, b2] = True
        # open the wall strip between maze cell (a, b) and (a2, b2); a is the x index
        if a2 != a:
            x = max(a, a2) * pitch
            img[b * pitch + wall:(b + 1) * pitch, x:x + wall] = 0
        else:
            y = max(b, b2) * pitch
            img[y:y + wall, a * pitch + wall:(a + 1) * pitch] = 0
        stack.append((a2, b2))
    return img


def soft_ramp(img: np.ndarray, width: float, peak: int) -> np.ndarray:
    """Soft cost near hard pixels: code round(peak (width - d) / width) for a
    Euclidean distance d < width to the nearest hard pixel (a distance
    transform of the hard image, Sec. VII)."""
    from scipy.ndimage import distance_transform_edt

    d = distance_transform_edt(img != HARD)
    soft = np.where(d < width, np.rint(peak * (width - d) / width), 0).astype(np.int32)
    out = np.where(img == HARD, HARD, np.clip(soft, 0, 254)).astype(np.uint8)
    return out


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def plain_64(seed: int = 1302) -> Scene:
    """64 x 64 cells x 64 headings, 8 random rectangles of side 3..12,
    vehicle 6 x 3, R = 10, N = 4, forward and reverse."""
    rng = np.random.default_rng(seed)
    n, nt = 64, 64
    veh = vehicle_box(6, 3)
    img = rect_clutter(rng, n, 8, 3, 12)
    start = sample_pose(rng, img, nt, veh)
    goal = sample_pose(rng, img, nt, veh)
    return Scene("plain_64", n, nt, 10.0, img, veh, start, goal, n_cycles=4, ct=uniform_ct(20),
                 half_cell=1, goal_radius=0, seed=seed)


def parking_256(seed: int = 1303) -> Scene:
    """Parallel parking, 256 x 256 cells x 256 headings at 0.05 m/cell: curb,
    two parked 4.5 x 1.8 m cars with a 6.5 m gap, ego 4.5 x 1.8 m, R = 5 m,
    N = 6, reverse gear at 1.5x."""
    n, nt = 256, 256
    img = np.zeros((n, n), np.uint8)
    img[:20, :] = HARD                      # curb
    img[24:60, 0:63] = HARD                 # parked car ending at x = 63
    img[24:60, 193:256] = HARD              # parked car starting at x = 193
    veh = vehicle_box(90, 36)
    return Scene("parking_256", n, nt, 100.0, img, veh, (150, 110, 0), (95, 42, 0), n_cycles=6,
                 ct=uniform_ct(200), gear=reverse_gear(384), half_cell=1, goal_radius=2,
                 seed=seed)


def maze_512(seed: int = 1304) -> Scene:
    """512 x 512 cells x 512 headings maze (16 x 16 maze cells, 28-cell
    corridors, 4-cell walls), vehicle 10 x 5, R = 12, soft ramp within 4 cells
    of walls, N = 20, start and goal at the centres of opposite corner cells.
    The start faces +x, the goal -x (180 degrees), a heading at which 20
    cycles reach the far corner of this maze."""
    rng = np.random.default_rng(seed)
    n_cells, pitch, wall = 16, 32, 4
    img = soft_ramp(maze(rng, n_cells, pitch, wall), 4.0, 64)
    c0 = wall + (pitch - wall) // 2
    c1 = (n_cells - 1) * pitch + c0
    return Scene("maze_512", 512, 512, 12.0, img, vehicle_box(10, 5), (c0, c0, 0), (c1, c1, 256),
                 n_cycles=20, ct=uniform_ct(24), half_cell=1, goal_radius=2, seed=seed)


def random_instance(rng, sides=(128, 256, 384), thetas=(128, 256), n_range=(4, 12),
                    len_range=(4, 12), occ=(0.05, 0.30), name="inst") -> Scene:
    """One planning instance of the batched workload."""
    n = int(rng.choice(sides))
    nt = int(rng.choice(thetas))
    img = mixed_clutter(rng, n, float(rng.uniform(*occ)))
    L = int(rng.integers(len_range[0], len_range[1] + 1))
    veh = vehicle_box(L, max(1, int(round(L / 2))))
    R = float(rng.integers(8, 21))
    start = sample_pose(rng, img, nt, veh)
    goal = sample_pose(rng, img, nt, veh)
    return Scene(name, n, nt, R, img, veh, start, goal,
                 n_cycles=int(rng.integers(n_range[0], n_range[1] + 1)), ct=uniform_ct(2 * R),
                 half_cell=1, goal_radius=2)


def batch_64(seed: int = 1305, count: int = 64) -> List[Scene]:
    """64 instances: sides from {128, 256, 384}, headings from {128, 256},
    5-30 % clutter, N in 4..12, vehicle length 4..12."""
    rng = np.random.default_rng(seed)
    return [random_instance(rng, name="batch%02d" % k) for k in range(count)]


def serving_requests(seed: int = 1306, count: int = 64, sides=(128, 256, 512, 1024),
                     thetas=(128, 256, 512)) -> List[Scene]:
    """Mixed serving requests: sides up to 1024, headings up to 512, 0-30 %
    clutter, N in 4..20."""
    rng = np.random.default_rng(seed)
    return [random_instance(rng, sides=sides, thetas=thetas, n_range=(4, 20), occ=(0.0, 0.30),
                            name="req%03d" % k) for k in range(count)]


def poisson_arrivals(seed: int, rate: float, count: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def free_space(n: int, nt: int, R: float, n_cycles: int, start=None, ct_cells: float = 0.0,
               schedule=DEFAULT_SCHEDULE, half_cell: int = 0, vehicle=(0, 0, 0)) -> Scene:
    """Empty scene (only the one-cell walls), for closed-form checks."""
    img = np.zeros((n, n), np.uint8)
    if start is None:
        start = (n // 2, n // 2, 0)
    return Scene("free_%d" % n, n, nt, R, img, tuple(vehicle), tuple(start), tuple(start), n_cycles,
                 ct=uniform_ct(ct_cells), schedule=tuple(schedule), half_cell=half_cell)


def random_small(seed: int, n: int = 32, nt: int = 32, R: float = 4.0, n_cycles: int = 3,
                 soft: bool = True, half_cell: int = 1, ct_cells: float = 3.0,
                 gear=None, schedule=DEFAULT_SCHEDULE, n_rect: int = 6) -> Scene:
    """Small random scene with hard rectangles and optionally random soft
    codes, for exhaustive checks."""
    rng = np.random.default_rng(seed)
    img = rect_clutter(rng, n, n_rect, 2, max(3, n // 6))
    if soft:
        s = rng.integers(0, 200, size=(n, n)).astype(np.uint8)
        s[rng.random((n, n)) < 0.5] = 0
        img = np.where(img == HARD, HARD, s).astype(np.uint8)
    veh = (1, 0, 0) if n >= 16 else (0, 0, 0)
    start = sample_pose(rng, img, nt, veh)
    goal = sample_pose(rng, img, nt, veh)
    if gear is None:
        gear = reverse_gear(int(rng.integers(256, 512)))
    ct = tuple(int(rng.integers(Q10, 6 * Q10)) for _ in range(6))
    return Scene("small_%d" % seed, n, nt, R, img, veh, start, goal, n_cycles, ct=ct,
                 gear=tuple(gear), schedule=tuple(schedule), half_cell=half_cell, seed=seed)


def reach_128(seed: int = 1307) -> Scene:
    """Maneuver-count reachability workload of App. C's timing table: 128 x
    128 cells x 512 headings, N = 8 maneuver cycles, hard obstacles only
    (axis-aligned rectangles, about 10 % of the area), vehicle 6 x 3, R = 10.
    The goal lies 3 cells along x and 24 against y from the start, turned
    by 180 degrees, like the example the paper solves with four maneuvers."""
    rng = np.random.default_rng(seed)
    n, nt = 128, 512
    veh = vehicle_box(6, 3)
    start, goal = (60, 80, 0), (63, 56, 256)
    img = rect_clutter(rng, n, 24, 4, 14)
    for (i, j, _t) in (start, goal):  # keep the end poses clear
        img[max(0, j - 8): j + 9, max(0, i - 8): i + 9] = 0
    return Scene("reach_128", n, nt, 10.0, img, veh, start, goal, n_cycles=8, ct=uniform_ct(10), half_cell=1,
                 goal_radius=0, seed=seed)


WORKLOADS = {
    "plain_64": plain_64,
    "parking_256": parking_256,
    "maze_512": maze_512,
    "reach_128": reach_128,
}
