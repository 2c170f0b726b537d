"""Pins of the oracle against the continuum vehicle with reverse gear (the
Reeds-Shepp car) in free space, within the error bounds the paper proves for
its graph (App. B): with the six maneuvers LF, SF, RB, RF, SB, LB at equal
gear the planner's vehicle is the Reeds-Shepp car of turn radius R, here
with a maneuver-counting transition cost d_T per maneuver at least the
sufficient one of App. B.

* Theorem 7 (the graph reaches what the continuum reaches): a configuration
  that some continuum path reaches at cost d (length plus d_T per maneuver)
  has a graph vertex within 7 + pi d / N_theta cells in x and y and 4
  headings whose value is at most d.  The continuum paths are drawn from the
  word shapes of Theorem 3 (CC|CC, C|CC|C, C|CC, CC|C, C|C S C, C S C|C,
  C|C|C, CSC, C|C S C|C, with cusps "|" reversing the gear) with random
  letters and segment lengths, and executed from the start: their end is
  reachable at their cost by construction, whether or not they are
  shortest, which is all the theorem asks.
* Corollary 2 / Theorem 6 (a graph path is a continuum path up to
  snapping): every back-tracked maneuver list, forward and reverse,
  executed exactly on circles of radius R and straight segments from the
  start, ends within m_c / 2 + m_s cells of the vertex the oracle reached
  (m_c turns, m_s straights) at the same heading, and its cost is d_T per
  maneuver plus the continuum length (up to the rounding of edge lengths to
  1/1024 cell) and at most the vertex's value.  With at most five
  maneuvers that end point is the X_C of Theorem 6, within 4 cells."""
import math

import numpy as np
import pytest

import oracle
from paper_2306_01301_amd import scenes
from tests.common import problem_of

TWO_PI = 2.0 * math.pi
LF, SF, RB, RF, SB, LB = oracle.LF, oracle.SF, oracle.RB, oracle.RF, oracle.SB, oracle.LB


def _execute(pose, segments, r):
    """Executes (letter, gear, amount) segments from pose (x, y, theta):
    letter 'L' / 'R' turns by an angle on the left / right circle of radius
    r, 'S' moves a distance along the heading; gear +1 forward, -1 reverse
    (reversing on a left circle turns the heading clockwise)."""
    x, y, th = pose
    for letter, gear, a in segments:
        if letter == "S":
            x, y = x + gear * a * math.cos(th), y + gear * a * math.sin(th)
        elif letter == "L":
            cx, cy = x - r * math.sin(th), y + r * math.cos(th)
            th = th + gear * a
            x, y = cx + r * math.sin(th), cy - r * math.cos(th)
        else:
            cx, cy = x + r * math.sin(th), y - r * math.cos(th)
            th = th - gear * a
            x, y = cx - r * math.sin(th), cy + r * math.cos(th)
    return x, y, th


def _cost(segments, r, d_t):
    length = sum(a if k == "S" else r * a for k, _, a in segments)
    return length + d_t * sum(1 for _, _, a in segments if a > 0.0)


def test_execution_closed_forms():
    """Reverse gear retraces forward motion; a full circle either way is the
    identity; a quarter turn forward then back returns."""
    r = 5.0
    p0 = (3.0, -2.0, 0.7)
    for letter in "LRS":
        a = 1.3 if letter != "S" else 7.5
        fwd = _execute(p0, [(letter, 1, a)], r)
        back = _execute(fwd, [(letter, -1, a)], r)
        assert max(abs(u - v) for u, v in zip(back, p0)) < 1e-12
    for letter in "LR":
        for gear in (1, -1):
            x, y, th = _execute(p0, [(letter, gear, TWO_PI)], r)
            assert abs(x - p0[0]) < 1e-12 and abs(y - p0[1]) < 1e-12
            assert abs(math.remainder(th - p0[2], TWO_PI)) < 1e-12
    # a forward left quarter turn from heading 0 ends at (r, r), heading 90 deg
    x, y, th = _execute((0.0, 0.0, 0.0), [("L", 1, math.pi / 2)], r)
    assert abs(x - r) < 1e-12 and abs(y - r) < 1e-12 and abs(th - math.pi / 2) < 1e-12
    # reversing a quarter of the right circle (centre (0, -r)) from heading 0
    # ends at (-r, -r), heading 90 deg
    x, y, th = _execute((0.0, 0.0, 0.0), [("R", -1, math.pi / 2)], r)
    assert abs(x + r) < 1e-12 and abs(y + r) < 1e-12 and abs(th - math.pi / 2) < 1e-12


# The word shapes of Theorem 3: per segment (letter kind, cusp before it);
# 'C' a circle, 'C2' a quarter circle, 'Cd' circles of one shared length,
# 'S' a straight.
SHAPES = [
    [("C", 0), ("Cd", 0), ("Cd", 1), ("C", 0)],            # C C_d | C_d C
    [("C", 0), ("Cd", 1), ("Cd", 0), ("C", 1)],            # C | C_d C_d | C
    [("C", 0), ("C", 1), ("C", 0)],                        # C | C C
    [("C", 0), ("C", 0), ("C", 1)],                        # C C | C
    [("C", 0), ("C2", 1), ("S", 0), ("C", 0)],             # C | C_pi/2 S C
    [("C", 0), ("S", 0), ("C2", 0), ("C", 1)],             # C S C_pi/2 | C
    [("C", 0), ("C", 1), ("C", 1)],                        # C | C | C
    [("C", 0), ("S", 0), ("C", 0)],                        # C S C
    [("C", 0), ("C2", 1), ("S", 0), ("C2", 0), ("C", 1)],  # C | C_pi/2 S C_pi/2 | C
]


def _random_word(rng, shape):
    gear = int(rng.choice((1, -1)))
    shared = float(rng.uniform(0.0, math.pi / 2))
    out = []
    for kind, cusp in shape:
        if cusp:
            gear = -gear
        if kind == "S":
            out.append(("S", gear, float(rng.uniform(0.0, 12.0))))
            continue
        letter = str(rng.choice(("L", "R")))
        a = {"C": float(rng.uniform(0.0, math.pi / 2)), "C2": math.pi / 2, "Cd": shared}[kind]
        out.append((letter, gear, a))
    return out


N, L, R = 96, 64, 6.0
START = (48, 48, 0)
CYCLES = 8
# App. B: d_T >= d_x + R d_theta + 4 R acos(1 - d_y / (4 R)) for one cell
D_T = math.ceil(1.0 + R * TWO_PI / L + 4 * R * math.acos(1.0 - 1.0 / (4 * R)))


@pytest.fixture(scope="module")
def solved():
    sc = scenes.free_space(N, L, R, CYCLES, start=START, ct_cells=D_T, half_cell=1)
    assert tuple(sc.schedule) == (LF, SF, RB, RF, SB, LB) and tuple(sc.gear) == (256,) * 6
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, 0, 0, 0)
    V = oracle.init(prob, B, START)
    oracle.cycles(prob, B, V, CYCLES)
    return prob, B, V, oracle.tables(prob)


def _represented(tb, i, j, T):
    """Point a vertex stands for with the half-cell representation (eq. 16)."""
    psi = tb["psi"]
    return i + 0.5 * psi[T], j + 0.5 * psi[(T + L // 4) % L]


def test_theorem_7_graph_reaches_the_reeds_shepp_set(solved):
    prob, B, V, tb = solved
    x0, y0 = _represented(tb, *START)
    rng = np.random.default_rng(2306)
    checked = 0
    for rep in range(12):
        for shape in SHAPES:
            word = _random_word(rng, shape)
            gx, gy, gth = _execute((x0, y0, 0.0), word, R)
            d = _cost(word, R, D_T)
            rad = 7.0 + math.pi * d / L
            ri = int(math.ceil(rad)) + 1
            centre = gth * L / TWO_PI
            best = oracle.INF
            for T in range(int(math.floor(centre - 4)), int(math.ceil(centre + 4)) + 1):
                if abs(T - centre) > 4:
                    continue
                TT = T % L
                i0, j0 = int(round(gx)), int(round(gy))
                ii, jj = np.meshgrid(np.arange(i0 - ri, i0 + ri + 1), np.arange(j0 - ri, j0 + ri + 1), indexing="xy")
                px, py = _represented(tb, ii, jj, TT)
                near = (np.abs(px - gx) <= rad) & (np.abs(py - gy) <= rad)
                vals = V[TT][jj[near] % N, ii[near] % N]
                best = min(best, int(vals.min()))
            edges = d * (L / (TWO_PI * R) + 1.0) + 10
            assert best <= 1024.0 * d + 0.5 * edges, (shape, word, d, best / 1024.0)
            checked += 1
    assert checked == 12 * len(SHAPES)


def _replay(tb, steps, start):
    """Executes back-tracked steps exactly: turns on circles of radius R
    (LF and RB raise the heading, RF and LB lower it), straights along or
    against the heading by steps / max(|cos|, |sin|)."""
    x0, y0 = _represented(tb, *start)
    pose = (x0, y0, TWO_PI * start[2] / L)
    length, n_edges, m_c, m_s = 0.0, 0, 0, 0
    for s in steps:
        th = pose[2]
        if s.maneuver in (SF, SB):
            seg = s.steps / max(abs(math.cos(th)), abs(math.sin(th)))
            pose = _execute(pose, [("S", 1 if s.maneuver == SF else -1, seg)], R)
            m_s += 1
        else:
            letter = "L" if s.maneuver in (LF, LB) else "R"
            gear = 1 if s.maneuver in (LF, RF) else -1
            seg = R * s.steps * TWO_PI / L
            pose = _execute(pose, [(letter, gear, s.steps * TWO_PI / L)], R)
            m_c += 1
        length += seg
        n_edges += s.steps
    return pose, length, n_edges, m_c, m_s


def test_corollary_2_backtracked_paths_are_reeds_shepp_paths(solved):
    prob, B, V, tb = solved
    rng = np.random.default_rng(11)
    checked = reversing = 0
    while checked < 80:
        i, j = (int(v) for v in rng.integers(START[0] - 18, START[0] + 19, size=2))
        T = int(rng.integers(0, L))
        if (i, j, T) == START or V[T, j, i] == oracle.INF:
            continue
        steps = oracle.backtrack(prob, B, V, START, (i, j, T))
        pose, length, n_edges, m_c, m_s = _replay(tb, steps, START)
        gx, gy = _represented(tb, i, j, T)
        snap = m_c / 2 + m_s
        assert abs(pose[0] - gx) <= snap + 1e-9 and abs(pose[1] - gy) <= snap + 1e-9, ((i, j, T), steps, pose)
        assert abs(math.remainder(pose[2] - TWO_PI * T / L, TWO_PI)) < 1e-9
        m = len(steps)
        if m <= 5:  # Theorem 6: the continuum end point is within 4 cells
            assert abs(pose[0] - gx) <= 4 and abs(pose[1] - gy) <= 4
        cost = sum(s.cost for s in steps)
        assert abs(cost - 1024 * D_T * m - 1024.0 * length) <= 0.5 * n_edges + 1e-6
        assert cost <= int(V[T, j, i])
        reversing += any(s.maneuver in (RB, SB, LB) for s in steps)
        checked += 1
    assert reversing >= 20  # the reverse gear is really exercised
