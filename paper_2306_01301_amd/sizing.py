"""Sizing rules of the paper, as plain formulas (no planner state).

* headings needed for collision checking and for unit turn steps (Sec. XIII);
* sufficient transition cost (App. B.C, the bound before Lemma 1);
* graph complexity and the kernel-style work count (Sec. XV, Tables 1-2);
* pose-cell updates and algorithmic HBM bytes of a plan on this library's
  data layout (uint32 values, uint8 obstacle codes).
"""
from __future__ import annotations

import math


def headings_for_collision(corner_distance: float, cell: float) -> float:
    """N_theta >= 2 pi d_c / d_x: one angular step moves a box corner less
    than one cell (Sec. XIII)."""
    return 2.0 * math.pi * corner_distance / cell


def headings_for_turns(turn_radius: float, cell: float) -> float:
    """N_theta >= 2 pi R / d_x: one turn edge moves less than one cell."""
    return 2.0 * math.pi * turn_radius / cell


def sufficient_transition_cost(dx: float, dy: float, dtheta: float, turn_radius: float) -> float:
    """d_T >= d_x + R d_theta + 4 R acos(1 - d_y / (4 R)): one transition
    cost pays for correcting one cell of error in each coordinate."""
    return dx + turn_radius * dtheta + 4.0 * turn_radius * math.acos(1.0 - dy / (4.0 * turn_radius))


GRAPHS = {  # (k_V, k_E), Sec. XV
    "piano": (1, 6),
    "compact": (3, 10),
    "star": (7, 18),
}


def graph_complexity(graph: str, n_r: float) -> float:
    """(k_V + k_E) log2(k_V N_R) N_R (Table 2), in units of N_R."""
    kv, ke = GRAPHS[graph]
    return (kv + ke) * math.log2(kv * n_r)


def kernel_complexity(n_cycles: int) -> int:
    """3 edge operations x 6 maneuvers x N_T cycles, in units of N_R."""
    return 18 * n_cycles


def memory_volumes(graph: str, kernel_style: bool = False) -> int:
    """Value plus heap memory in volumes of N_R entries (Table 1)."""
    if kernel_style:
        return 1
    kv, _ = GRAPHS[graph]
    return 3 * kv


def pose_updates(nx: int, nt: int, n_cycles: int, n_sched: int = 6) -> int:
    """Vertices relaxed by a plan: every scheduled sweep relaxes every pose once."""
    return n_sched * n_cycles * nx * nx * nt


BYTES_PER_UPDATE = 9  # read value (4 B) + read obstacle code (1 B) + write value (4 B)


def sweep_bytes(nx: int, nt: int, n_cycles: int, n_sched: int = 6) -> int:
    return BYTES_PER_UPDATE * pose_updates(nx, nt, n_cycles, n_sched)


def admission_bytes(nx: int, nt: int) -> int:
    """Admission footprint of a request: 3 vertices x 2 gears x 4 B per pose
    plus the 1 B collision volume."""
    return 25 * nx * nx * nt
