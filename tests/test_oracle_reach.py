"""Pins of the oracle's maneuver-count reachability (App. C, Insert 2)
against a second route to the same sets: breadth-first search over the
explicit successor maps of eqs. (25)-(31), where one maneuver is any number
of successor steps of one maneuver through free vertices.  Also: every
cycle uses the previous volume only (the schedule order cannot matter), the
cost sweeps reach at least as much in as many cycles, goal search is the
brute-force minimum, and every back-tracked path replays through the
explicit graph."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2306_01301_amd import scenes
from tests.common import cell, problem_of
from tests.pins import graph as G

HARD = 255
LF, SF, RB, RF, SB, LB = range(6)


def _hard_only(img):
    return np.where(img == HARD, HARD, 0).astype(np.uint8)


def _setup(sc):
    prob = problem_of(sc)
    B = oracle.render(prob, _hard_only(sc.image), *sc.vehicle)
    g = G.Graph(sc.nx, sc.nt, oracle.tables(prob), B, sc.ct)
    return prob, B, g


def bfs_levels(g, B, start, schedule, n_cycles):
    """Level m = fewest maneuvers: R_{m+1} adds, for every scheduled
    maneuver, the vertices reached from R_m by following that maneuver's
    successors through free vertices."""
    free = B.reshape(-1) != HARD
    NR = free.size
    level = np.full(NR, 255, np.uint8)
    R = np.zeros(NR, bool)
    R[start] = True
    level[start] = 0
    for m in range(n_cycles):
        nxt = R.copy()
        for mu in sorted(set(schedule)):
            got = R.copy()
            frontier = R.copy()
            while True:
                nb = np.zeros(NR, bool)
                nb[g.succ[mu][np.nonzero(frontier)[0]]] = True
                nb &= free & ~got
                if not nb.any():
                    break
                got |= nb
                frontier = nb
            nxt |= got
        level[nxt & (level == 255)] = m + 1
        R = nxt
    return level.reshape(B.shape)


CASES = [
    (1, 16, 16, 2.0, scenes.DEFAULT_SCHEDULE, 3),
    (2, 24, 24, 3.0, scenes.DEFAULT_SCHEDULE, 4),
    (3, 24, 16, 3.0, scenes.FORWARD_SCHEDULE, 4),
    (4, 32, 32, 4.0, (LF, SB, RB), 3),
    (5, 32, 24, 3.5, scenes.DEFAULT_SCHEDULE, 5),
]


@pytest.mark.parametrize("seed,n,nt,R,sched,ncyc", CASES)
def test_levels_equal_breadth_first_search(seed, n, nt, R, sched, ncyc):
    sc = scenes.random_small(seed, n=n, nt=nt, R=R, schedule=sched)
    prob, B, g = _setup(sc)
    level = oracle.reach(prob, B, sc.start, ncyc)
    want = bfs_levels(g, B, cell(n, *sc.start), sched, ncyc)
    assert np.array_equal(level, want)
    # levels are nested and only free vertices are reached
    assert np.all(level[B == HARD] == 255)
    assert level.reshape(-1)[cell(n, *sc.start)] == 0
    assert (level == 0).sum() == 1


def test_schedule_order_does_not_matter():
    sc = scenes.random_small(6, n=24, nt=24, R=3.0)
    prob, B, _ = _setup(sc)
    base = oracle.reach(prob, B, sc.start, 3)
    for perm in [(5, 4, 3, 2, 1, 0), (1, 4, 0, 2, 3, 5)]:
        p2 = problem_of(sc.with_(schedule=perm))
        assert np.array_equal(oracle.reach(p2, B, sc.start, 3), base)


def test_cost_sweeps_reach_at_least_as_much():
    """In-place cost sweeps see every earlier sweep of the cycle, so after n
    cycles every vertex of level <= n has a finite value."""
    sc = scenes.random_small(7, n=32, nt=32, R=4.0)
    prob, B, _ = _setup(sc)
    level = oracle.reach(prob, B, sc.start, 3)
    V = oracle.init(prob, B, sc.start)
    oracle.cycles(prob, B, V, 3)
    assert np.all(V[level <= 3] != oracle.INF)


def test_zero_cycles_and_errors():
    sc = scenes.random_small(8, n=16, nt=8, R=1.5)
    prob, B, _ = _setup(sc)
    level = oracle.reach(prob, B, sc.start, 0)
    assert (level != 255).sum() == 1
    hard = tuple(int(v) for v in np.argwhere(B == HARD)[0][::-1])  # (i, j, T)
    with pytest.raises(oracle.OracleError):
        oracle.reach(prob, B, hard, 2)
    with pytest.raises(oracle.OracleError):
        oracle.reach(prob, B, sc.start, 255)


def _brute_goal(level, goal, d):
    L, N, _ = level.shape
    best = None
    for dt, dy, dx in itertools.product(range(-d, d + 1), repeat=3):
        i, j, T = (goal[0] + dx) % N, (goal[1] + dy) % N, (goal[2] + dt) % L
        lv = int(level[T, j, i])
        if lv == 255:
            continue
        key = (lv, abs(dx) + abs(dy) + abs(dt), dt, dy, dx)
        if best is None or key < best[0]:
            best = (key, (i, j, T))
    return best


@pytest.mark.parametrize("seed", [11, 12, 13, 14])
def test_goal_and_backtrack_replay(seed):
    sc = scenes.random_small(seed, n=32, nt=32, R=4.0)
    prob, B, g = _setup(sc)
    level = oracle.reach(prob, B, sc.start, 5)
    for d in (0, 2):
        want = _brute_goal(level, sc.goal, d)
        if want is None:
            with pytest.raises(oracle.OracleError):
                oracle.reach_goal(prob, level, sc.goal, d)
            continue
        best, lv = oracle.reach_goal(prob, level, sc.goal, d)
        assert (best, lv) == (want[1], want[0][0])
        steps = oracle.reach_backtrack(prob, B, level, best)
        assert len(steps) == lv
        x = cell(sc.nx, *sc.start)
        free = B.reshape(-1) != HARD
        for k, s in enumerate(steps):
            assert cell(sc.nx, *s.frm) == x
            assert level.reshape(-1)[x] == k
            for _ in range(s.steps):
                x = int(g.succ[s.maneuver][x])
                assert free[x]
            assert cell(sc.nx, *s.to) == x
            assert s.maneuver in sc.schedule and s.cost == 1
        assert x == cell(sc.nx, *best)
