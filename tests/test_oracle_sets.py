"""Pins of the oracle's start sets and goal sets (Sec. III.A: a set of start
states with costs and a set of goal states with rewards; Sec. IX: the goal
criterion; Sec. XII: a maneuver already in progress continues without a
transition cost).  At convergence the swept values equal Dijkstra on the
Star graph from the same sources (an independent code route); a goal
window equals the goal set of its poses with the window's penalties; and
every back-tracked plan replays through the explicit graph."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2306_01301_amd import scenes
from tests.common import cell, problem_of
from tests.pins import graph as G

INF = oracle.INF
HARD = 255


def _setup(sc):
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    g = G.Graph(sc.nx, sc.nt, oracle.tables(prob), B, sc.ct)
    return prob, B, g


def _free_poses(rng, B, count):
    free = np.argwhere(B != HARD)
    pick = free[rng.choice(len(free), size=count, replace=False)]
    return [(int(i), int(j), int(T)) for T, j, i in pick]


def test_single_start_at_rest_equals_init():
    sc = scenes.random_small(3, n=24, nt=16, R=3.0)
    prob, B, _ = _setup(sc)
    V1 = oracle.init(prob, B, sc.start)
    V2 = oracle.init_set(prob, B, [(*sc.start, 0)])
    assert np.array_equal(V1, V2)
    oracle.cycles(prob, B, V1, 3)
    oracle.cycles(prob, B, V2, 3)
    assert np.array_equal(V1, V2)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_start_sets_converge_to_dijkstra(seed):
    rng = np.random.default_rng(seed)
    sc = scenes.random_small(40 + seed, n=16, nt=16, R=2.0)
    prob, B, g = _setup(sc)
    N = sc.nx
    poses = _free_poses(rng, B, 3)
    starts = [(*poses[0], 0), (*poses[1], int(rng.integers(0, 20000)), int(sc.schedule[2])),
              (*poses[2], int(rng.integers(0, 20000)), -1)]
    V = oracle.init_set(prob, B, starts)
    oracle.cycles(prob, B, V, 40)
    src = [(cell(N, *s[:3]), s[3], s[4] if len(s) > 4 else -1) for s in starts]
    want = G.star_dijkstra_sources(g, sc.schedule, src)
    assert np.array_equal(V.reshape(-1).astype(np.int64), want)


def test_maneuver_in_progress_outside_the_schedule():
    """The in-progress maneuver need not be scheduled: its curve is seeded
    once, and the scheduled maneuvers continue from there."""
    sc = scenes.random_small(51, n=16, nt=16, R=2.0, schedule=scenes.FORWARD_SCHEDULE)
    prob, B, g = _setup(sc)
    start = (*sc.start, 500, oracle.SB)
    V = oracle.init_set(prob, B, [start])
    oracle.cycles(prob, B, V, 40)
    want = G.star_dijkstra_sources(g, sc.schedule, [(cell(sc.nx, *sc.start), 500, oracle.SB)])
    assert np.array_equal(V.reshape(-1).astype(np.int64), want)


def test_goal_window_equals_goal_set():
    sc = scenes.random_small(61, n=32, nt=32, R=4.0)
    prob, B, _ = _setup(sc)
    V = oracle.init(prob, B, sc.start)
    oracle.cycles(prob, B, V, 3)
    N, L = sc.nx, sc.nt
    for d, wxy, wt in ((0, 0, 0), (2, 300, 700), (3, 1024, 0)):
        keyed = []
        for dt, dy, dx in itertools.product(range(-d, d + 1), repeat=3):
            pose = ((sc.goal[0] + dx) % N, (sc.goal[1] + dy) % N, (sc.goal[2] + dt) % L)
            pen = wxy * (abs(dx) + abs(dy)) + wt * abs(dt)
            keyed.append(((abs(dx) + abs(dy) + abs(dt), dt, dy, dx), pose, pen))
        keyed.sort()
        goals = [p for _, p, _ in keyed]
        pens = [q for _, _, q in keyed]
        try:
            want = oracle.goal_search(prob, B, V, sc.goal, d, wxy, wt)
        except oracle.OracleError:
            with pytest.raises(oracle.OracleError):
                oracle.goal_set(prob, B, V, goals, pens)
            continue
        k, score = oracle.goal_set(prob, B, V, goals, pens)
        assert (goals[k], score) == want


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_set_backtracking_replays(seed):
    rng = np.random.default_rng(seed)
    sc = scenes.random_small(70 + seed, n=24, nt=24, R=3.0)
    prob, B, g = _setup(sc)
    N = sc.nx
    poses = _free_poses(rng, B, 4)
    starts = [(*poses[0], 0, -1), (*poses[1], 3000, int(sc.schedule[1])), (*poses[2], 1500, oracle.LF)]
    V = oracle.init_set(prob, B, starts)
    oracle.cycles(prob, B, V, 30)
    goal = poses[3]
    if V[goal[2], goal[1], goal[0]] == INF:
        pytest.skip("goal unreached")
    steps = oracle.backtrack_set(prob, B, V, starts, goal)
    first = cell(N, *steps[0].frm) if steps else cell(N, *goal)
    x = first
    for k, s in enumerate(steps):
        assert cell(N, *s.frm) == x
        E = 0
        for _ in range(s.steps):
            E += int(g.w[s.maneuver][x])
            x = int(g.succ[s.maneuver][x])
        assert cell(N, *s.to) == x
        in_progress = k == 0 and any(cell(N, *t[:3]) == first and t[4] == s.maneuver and t[4] >= 0 and
                                     t[3] + E == int(V.reshape(-1)[x]) for t in starts) and s.cost == E
        assert s.cost == E + (0 if in_progress else g.ct[s.maneuver])
    assert x == cell(N, *goal)
    # the plan's total cost: the start cost plus the step costs, equal to V(goal) at convergence
    starts_at = [t for t in starts if cell(N, *t[:3]) == first]
    assert any(t[3] + sum(s.cost for s in steps) == int(V[goal[2], goal[1], goal[0]]) for t in starts_at)
