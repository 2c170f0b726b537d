"""Pins of the oracle against the continuum forward-only vehicle (Dubins) in
free space, within the error bounds the paper proves for its graph
(App. B): with the forward maneuvers LF, SF, RF the planner's vehicle is
the Dubins car of turn radius R, here with a maneuver-counting transition
cost d_T per maneuver at least the sufficient one of App. B.

* Theorem 7 (graph reaches what the continuum reaches): for a goal that a
  Dubins word reaches at cost d (length plus d_T per maneuver), some vertex
  within 7 + pi d / N_theta cells in x and y and 4 headings of the goal has
  a value of at most d.
* Corollary 2 (a graph path is a continuum path up to snapping): the
  back-tracked maneuver list, executed exactly on circles of radius R and
  straight segments from the start, ends within ceil(3m/2)/2 cells of the
  vertex the oracle reached (m maneuvers), at the same heading; its cost is
  d_T m plus the continuum length (up to the rounding of the edge lengths
  to 1/1024 cell) and at most the vertex's value; and that length is at
  least the Dubins distance to where it ends.

The Dubins distance below is the minimum over the six words LSL, RSR,
LSR, RSL, RLR, LRL, each built from tangent circles; every candidate path
is executed and must end at its target, which checks the construction."""
import math

import numpy as np
import pytest

import oracle
from paper_2306_01301_amd import scenes
from tests.common import problem_of

TWO_PI = 2.0 * math.pi
LF, SF, RF = oracle.LF, oracle.SF, oracle.RF


def _m2pi(a):
    return a % TWO_PI


def _left_center(x, y, th, r):
    return (x - r * math.sin(th), y + r * math.cos(th))


def _right_center(x, y, th, r):
    return (x + r * math.sin(th), y - r * math.cos(th))


def _run(pose, segments, r):
    """Executes (kind, amount) segments: 'L'/'R' turn by an angle, 'S' moves
    a distance along the heading."""
    x, y, th = pose
    for kind, a in segments:
        if kind == "S":
            x, y = x + a * math.cos(th), y + a * math.sin(th)
        elif kind == "L":
            cx, cy = _left_center(x, y, th, r)
            th = th + a
            x, y = cx + r * math.sin(th), cy - r * math.cos(th)
        else:
            cx, cy = _right_center(x, y, th, r)
            th = th - a
            x, y = cx - r * math.sin(th), cy + r * math.cos(th)
    return x, y, th


def _heading_on(kind, p, c):
    """Heading of forward motion at point p of a circle with centre c."""
    dx, dy = p[0] - c[0], p[1] - c[1]
    return math.atan2(dx, -dy) if kind == "L" else math.atan2(-dx, dy)


def _arc(kind, a, b):
    """Turning angle from heading a to heading b on a left or right circle."""
    return _m2pi(b - a) if kind == "L" else _m2pi(a - b)


def dubins(start, goal, r, transition=0.0):
    """Shortest length over the six words; with `transition` > 0, the
    smallest length plus `transition` per non-empty segment instead."""
    x0, y0, t0 = start
    x1, y1, t1 = goal
    centers = {"L": (_left_center(x0, y0, t0, r), _left_center(x1, y1, t1, r)),
               "R": (_right_center(x0, y0, t0, r), _right_center(x1, y1, t1, r))}
    cands = []
    for a in "LR":
        for b in "LR":
            c0, c1 = centers[a][0], centers[b][1]
            vx, vy = c1[0] - c0[0], c1[1] - c0[1]
            D = math.hypot(vx, vy)
            if a == b:
                phi, ell = math.atan2(vy, vx), D
            else:
                if D < 2 * r:
                    continue
                ell = math.sqrt(max(D * D - 4 * r * r, 0.0))
                tilt = math.atan2(2 * r, ell)
                phi = math.atan2(vy, vx) + (tilt if a == "L" else -tilt)
            cands.append([(a, _arc(a, t0, phi)), ("S", ell), (b, _arc(b, phi, t1))])
    for a, m in (("L", "R"), ("R", "L")):
        c0, c1 = centers[a][0], centers[a][1]
        vx, vy = c1[0] - c0[0], c1[1] - c0[1]
        D = math.hypot(vx, vy)
        if D > 4 * r or D == 0.0:
            continue
        h = math.sqrt(max(4 * r * r - D * D / 4, 0.0))
        for sgn in (1, -1):
            c2 = ((c0[0] + c1[0]) / 2 - sgn * h * vy / D, (c0[1] + c1[1]) / 2 + sgn * h * vx / D)
            p1 = ((c0[0] + c2[0]) / 2, (c0[1] + c2[1]) / 2)
            p2 = ((c2[0] + c1[0]) / 2, (c2[1] + c1[1]) / 2)
            h1, h2 = _heading_on(a, p1, c0), _heading_on(a, p2, c1)
            cands.append([(a, _arc(a, t0, h1)), (m, _arc(m, h1, h2)), (a, _arc(a, h2, t1))])
    best = math.inf
    for segs in cands:
        x, y, th = _run(start, segs, r)
        ok = math.hypot(x - x1, y - y1) < 1e-7 and abs(math.remainder(th - t1, TWO_PI)) < 1e-7
        assert ok, segs  # every constructed word must reach the goal
        length = sum(v if k == "S" else r * v for k, v in segs)
        maneuvers = sum(1 for k, v in segs if v > 1e-12)
        best = min(best, length + transition * maneuvers)
    return best


def test_dubins_construction():
    """Closed forms: straight ahead, a U-turn, a full-circle return."""
    r = 3.0
    assert abs(dubins((0, 0, 0), (10, 0, 0), r) - 10.0) < 1e-9
    assert abs(dubins((0, 0, 0), (0, 2 * r, math.pi), r) - math.pi * r) < 1e-9
    rng = np.random.default_rng(5)
    for _ in range(300):
        a = (0.0, 0.0, rng.uniform(0, TWO_PI))
        b = (rng.uniform(-15, 15), rng.uniform(-15, 15), rng.uniform(0, TWO_PI))
        m = (rng.uniform(-15, 15), rng.uniform(-15, 15), rng.uniform(0, TWO_PI))
        d = dubins(a, b, r)
        assert d >= math.hypot(b[0], b[1]) - 1e-9
        assert d <= dubins(a, m, r) + dubins(m, b, r) + 1e-7  # triangle inequality


N, L, R = 96, 64, 6.0
START = (48, 48, 0)
CYCLES = 8
# App. B: d_T >= d_x + R d_theta + 4 R acos(1 - d_y / (4 R)) for one cell
D_T = math.ceil(1.0 + R * TWO_PI / L + 4 * R * math.acos(1.0 - 1.0 / (4 * R)))


@pytest.fixture(scope="module")
def solved():
    sc = scenes.free_space(N, L, R, CYCLES, start=START, ct_cells=D_T, schedule=scenes.FORWARD_SCHEDULE,
                           half_cell=1)
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, 0, 0, 0)
    V = oracle.init(prob, B, START)
    oracle.cycles(prob, B, V, CYCLES)
    return prob, B, V, oracle.tables(prob)


def _represented(tb, i, j, T):
    """Point a vertex stands for with the half-cell representation (eq. 16)."""
    psi = tb["psi"]
    return i + 0.5 * psi[T], j + 0.5 * psi[(T + L // 4) % L]


def _goals(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        i, j = (int(v) for v in rng.integers(START[0] - 20, START[0] + 21, size=2))
        T = int(rng.integers(0, L))
        if (i, j, T) != START:
            out.append((i, j, T))
    return out


def test_theorem_7_graph_reaches_the_dubins_set(solved):
    prob, B, V, tb = solved
    x0 = _represented(tb, *START)
    for goal in _goals(60, 7):
        i, j, T = goal
        gx, gy = _represented(tb, i, j, T)
        d = dubins((x0[0], x0[1], 0.0), (gx, gy, TWO_PI * T / L), R, transition=D_T)
        rad = 7.0 + math.pi * d / L
        ri = int(math.floor(rad))
        win = []
        for dt in range(-4, 5):
            TT = (T + dt) % L
            sl = V[TT, max(0, j - ri - 1): j + ri + 2, max(0, i - ri - 1): i + ri + 2]
            jj, ii = np.meshgrid(np.arange(max(0, j - ri - 1), j + ri + 2), np.arange(max(0, i - ri - 1), i + ri + 2),
                                 indexing="ij")
            px, py = _represented(tb, ii, jj, TT)
            near = (np.abs(px - gx) <= rad) & (np.abs(py - gy) <= rad)
            win.append(sl[near].min())
        edges = d * (L / (TWO_PI * R) + 1.0) + 8
        assert min(win) <= 1024.0 * d + 0.5 * edges, (goal, d, min(win) / 1024.0)


def test_corollary_2_backtracked_paths_are_continuum_paths(solved):
    prob, B, V, tb = solved
    x0 = _represented(tb, *START)
    checked = 0
    for goal in _goals(60, 8):
        i, j, T = goal
        if V[T, j, i] == oracle.INF:
            continue
        steps = oracle.backtrack(prob, B, V, START, goal)
        pose = (x0[0], x0[1], 0.0)
        length, n_edges = 0.0, 0
        for s in steps:
            th = pose[2]
            if s.maneuver == SF:
                seg = s.steps / max(abs(math.cos(th)), abs(math.sin(th)))
                pose = _run(pose, [("S", seg)], R)
            else:
                seg = R * s.steps * TWO_PI / L
                pose = _run(pose, [("L" if s.maneuver == LF else "R", s.steps * TWO_PI / L)], R)
            length += seg
            n_edges += s.steps
        m = len(steps)
        gx, gy = _represented(tb, i, j, T)
        snap = math.ceil(3 * m / 2) / 2
        assert abs(pose[0] - gx) <= snap + 1e-9 and abs(pose[1] - gy) <= snap + 1e-9, (goal, m, pose, (gx, gy))
        assert abs(math.remainder(pose[2] - TWO_PI * T / L, TWO_PI)) < 1e-9
        cost = sum(s.cost for s in steps)
        assert abs(cost - 1024 * D_T * m - 1024.0 * length) <= 0.5 * n_edges + 1e-6
        assert cost <= int(V[T, j, i])
        assert dubins((x0[0], x0[1], 0.0), pose, R) <= length + 1e-7
        checked += 1
    assert checked >= 50
