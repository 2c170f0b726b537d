"""Pins of the oracle's maneuver sweeps (Sec. VIII.B, Insert 1) against the
explicit graph of eqs. (25)-(31): one sweep equals the fixed point of its
maneuver's edges (at every N, exactly), N cycles at convergence equal
Dijkstra on the Star graph (Sec. V.A), one cycle equals the brute-force
minimum over all paths whose maneuvers follow the cycle order
(Sec. XVI.A), and closed forms in free space."""
import numpy as np
import pytest

import oracle
from paper_2306_01301_amd import scenes
from tests.common import cell, problem_of
from tests.pins import graph as G

INF = oracle.INF


def _setup(sc):
    prob = problem_of(sc)
    f, r, s = sc.vehicle
    B = oracle.render(prob, sc.image, f, r, s)
    V = oracle.init(prob, B, sc.start)
    g = G.Graph(sc.nx, sc.nt, oracle.tables(prob), B, sc.ct)
    return prob, B, V, g


@pytest.mark.parametrize("seed,hc", [(1, 1), (2, 0), (3, 1), (4, 1)])
def test_each_sweep_equals_explicit_fixed_point(seed, hc):
    sc = scenes.random_small(seed, n=24, nt=24, R=3.0, half_cell=hc)
    prob, B, V, g = _setup(sc)
    for n in range(3):
        for mu in sc.schedule:
            want = G.schedule_dp_sweep(g, mu, V)
            oracle.sweep(prob, mu, B, V)
            assert np.array_equal(V, want), (n, oracle.NAMES[mu])


def test_sweep_on_random_values_equals_explicit_fixed_point():
    """The same on arbitrary pre-sweep values (not reachable from one
    start), including values close to saturation."""
    sc = scenes.random_small(9, n=20, nt=16, R=2.5)
    prob, B, _, g = _setup(sc)
    rng = np.random.default_rng(5)
    for mu in range(6):
        V = rng.integers(0, 1 << 20, size=B.shape, dtype=np.uint64).astype(np.uint32)
        V[rng.random(B.shape) < 0.3] = INF
        V[rng.random(B.shape) < 0.05] = INF - rng.integers(1, 5000)
        V[B == 255] = INF
        want = G.schedule_dp_sweep(g, mu, V)
        oracle.sweep(prob, mu, B, V)
        assert np.array_equal(V, want), oracle.NAMES[mu]


@pytest.mark.parametrize("seed,sched", [(11, scenes.DEFAULT_SCHEDULE), (12, scenes.DEFAULT_SCHEDULE),
                                        (13, scenes.FORWARD_SCHEDULE)])
def test_convergence_equals_star_dijkstra(seed, sched):
    sc = scenes.random_small(seed, n=20, nt=16, R=2.5, schedule=sched)
    prob, B, V, g = _setup(sc)
    prev = None
    for n in range(200):
        oracle.cycles(prob, B, V, 1)
        if prev is not None and np.array_equal(prev, V):
            break
        prev = V.copy()
    else:
        pytest.fail("no convergence")
    d = G.star_dijkstra(g, sched, cell(sc.nx, *sc.start))
    hard = B.reshape(-1) == 255
    assert np.array_equal(V.reshape(-1)[~hard], d[~hard])
    assert np.all(V.reshape(-1)[hard] == INF)


def test_star_equals_compact_when_costs_conform():
    """Sec. V.A: with no straight transition cost and equal costs for the
    forward and backward versions, the Compact graph has the same distances."""
    sc = scenes.random_small(21, n=16, nt=16, R=2.0)
    ct = [3000, 0, 2500, 2500, 0, 3000]
    sc = sc.with_(ct=tuple(ct))
    prob, B, V, g = _setup(sc)
    s = cell(sc.nx, *sc.start)
    d_star = G.star_dijkstra(g, sc.schedule, s)
    d_comp = G.compact_dijkstra(g, s, 3000, 2500)
    assert np.array_equal(d_star, d_comp)


@pytest.mark.parametrize("seed,hc", [(31, 1), (32, 0)])
def test_one_cycle_equals_brute_force(seed, hc):
    """Every path whose maneuvers are a sub-sequence of one cycle, with every
    step count, enumerated explicitly (8^6 paths)."""
    sc = scenes.random_small(seed, n=8, nt=8, R=1.5, half_cell=hc, n_rect=1)
    prob, B, V, g = _setup(sc)
    oracle.cycles(prob, B, V, 1)
    steps = {mu: 7 for mu in range(6)}
    best = G.enumerate_paths(g, cell(sc.nx, *sc.start), list(sc.schedule), steps)
    hard = B.reshape(-1) == 255
    assert np.array_equal(V.reshape(-1)[~hard], best[~hard])


def test_three_cycles_cover_every_three_maneuver_plan():
    """Sec. XVI.A: N cycles evaluate all N-maneuver plans in any order."""
    sc = scenes.random_small(41, n=10, nt=8, R=1.5, n_rect=2)
    prob, B, V, g = _setup(sc)
    oracle.cycles(prob, B, V, 3)
    steps = {mu: 9 for mu in range(6)}
    start = cell(sc.nx, *sc.start)
    rng = np.random.default_rng(0)
    seqs = [tuple(rng.integers(0, 6, 3)) for _ in range(25)]
    free = B.reshape(-1) != 255
    for seq in seqs:
        best = G.enumerate_paths(g, start, list(seq), steps)
        assert np.all(V.reshape(-1).astype(np.int64)[free] <= best[free]), seq


def test_free_space_closed_forms():
    """A pure straight of k cells costs ct + k Lq (free-space slowness 1);
    a pure turn of m edges costs ct + m Lq_turn and lands where eq. (18)
    says; a reversing gear scales the edge sum."""
    N, L, R = 64, 64, 8.0
    ct = 60 * 1024  # larger than any detour, so single maneuvers are optimal
    gear = [256, 256, 384, 256, 384, 384]
    sc = scenes.free_space(N, L, R, 1, start=(20, 32, 0), ct_cells=60, half_cell=0).with_(gear=tuple(gear))
    prob, B, V, g = _setup(sc)
    oracle.cycles(prob, B, V, 1)
    tb = oracle.tables(prob)
    for k in range(1, 30):
        assert V[0, 32, 20 + k] == ct + k * int(tb["Lq"][oracle.SF, 0])
    for k in range(1, 15):
        assert V[0, 32, 20 - k] == ct + k * int(tb["Lq"][oracle.SB, 0])
    assert tb["Lq"][oracle.SB, 0] == 1536 and tb["Lq"][oracle.SF, 0] == 1024
    beta = tb["beta"]
    xp, yp = 20 - beta[0], 32 - beta[3 * L // 4]
    for m in range(1, 12):
        i, j = xp + beta[m], yp + beta[(m + 3 * L // 4) % L]
        assert V[m, j, i] == ct + m * int(tb["Lq"][oracle.LF, 0])


def test_values_never_increase_with_more_cycles():
    sc = scenes.random_small(51, n=24, nt=24, R=3.0)
    prob, B, V, g = _setup(sc)
    prev = V.copy()
    for _ in range(4):
        oracle.cycles(prob, B, V, 1)
        assert np.all(V <= prev)
        prev = V.copy()


def test_resume_equals_one_run():
    sc = scenes.random_small(52, n=24, nt=24, R=3.0)
    prob, B, V, g = _setup(sc)
    V2 = V.copy()
    oracle.cycles(prob, B, V, 5)
    oracle.cycles(prob, B, V2, 2)
    oracle.cycles(prob, B, V2, 3)
    assert np.array_equal(V, V2)


def _transpose_scene(sc):
    """Reflect across the diagonal: (i, j, theta) -> (j, i, pi/2 - theta).
    Left and right turns swap; straights keep their direction."""
    L = sc.nt
    swap = {oracle.LF: oracle.RF, oracle.RF: oracle.LF, oracle.LB: oracle.RB, oracle.RB: oracle.LB,
            oracle.SF: oracle.SF, oracle.SB: oracle.SB}
    ct = [0] * 6
    gear = [0] * 6
    for mu in range(6):
        ct[swap[mu]] = sc.ct[mu]
        gear[swap[mu]] = sc.gear[mu]
    i, j, T = sc.start
    return sc.with_(image=np.ascontiguousarray(sc.image.T), start=(j, i, (L // 4 - T) % L),
                    schedule=tuple(swap[m] for m in sc.schedule), ct=tuple(ct), gear=tuple(gear))


@pytest.mark.parametrize("seed", [61, 62])
def test_mirror_symmetry(seed):
    """With plain rounding the tables are exactly symmetric, so the value
    volume of the reflected scene is the reflected value volume."""
    sc = scenes.random_small(seed, n=24, nt=24, R=3.0, half_cell=0).with_(vehicle=(3, 1, 1))
    prob, B, V, g = _setup(sc)
    oracle.cycles(prob, B, V, 3)
    sc2 = _transpose_scene(sc)
    prob2, B2, V2, g2 = _setup(sc2)
    oracle.cycles(prob2, B2, V2, 3)
    L = sc.nt
    T = np.arange(L)
    Bm = np.transpose(B, (0, 2, 1))[(L // 4 - T) % L]
    Vm = np.transpose(V, (0, 2, 1))[(L // 4 - T) % L]
    assert np.array_equal(B2, Bm)
    assert np.array_equal(V2, Vm)
