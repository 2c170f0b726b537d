"""GPU parity: every stage of the HIP path against the CPU oracle, element by
element, bit-exact (integer costs and codes), through the C ABI.

Sizes span several tiles and ragged tails (N not a multiple of 64, curve
lengths not a multiple of the section size, non-power-of-two grids) and the
paper-shaped workloads; the largest cases run at full size."""
import os
import sys
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2306_01301_amd import scenes
from paper_2306_01301_amd import planner as P
from tests.common import problem_of

pytestmark = pytest.mark.gpu

INF = 0xFFFFFFFF


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()  # raises if the library is missing
    oracle.set_threads(min(16, os.cpu_count() or 1))


def _planner(sc):
    return P.planner_for(sc)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


TABLE_CASES = [(64, 64, 10.0, 1), (64, 64, 10.0, 0), (64, 64, 3.0, 1), (40, 24, 3.0, 1), (256, 256, 100.0, 1), (512, 512, 12.0, 1),
               (384, 128, 15.0, 1), (200, 72, 7.5, 0), (1024, 512, 80.0, 1)]


@pytest.mark.parametrize("N,L,R,hc", TABLE_CASES)
def test_tables_match_oracle(N, L, R, hc):
    gear = (256, 256, 384, 256, 384, 384)
    sc = scenes.free_space(N, L, R, 1, half_cell=hc).with_(gear=gear, ct=scenes.uniform_ct(3))
    note("tables %s" % ((N, L, R, hc),))
    p = _planner(sc)
    got = p.tables()
    want = oracle.tables(problem_of(sc))
    for k in want:
        assert np.array_equal(got[k], want[k]), k
    p.close()


RENDER_CASES = [
    ("plain_64", lambda: scenes.plain_64()),
    ("small40_hc", lambda: scenes.random_small(3, n=40, nt=24, R=3.0).with_(vehicle=(5, 2, 2))),
    ("small48_plain", lambda: scenes.random_small(4, n=48, nt=32, R=4.0, half_cell=0).with_(vehicle=(7, 1, 3))),
    ("clutter200", lambda: scenes.random_instance(np.random.default_rng(7), sides=(200,), thetas=(72,))),
    ("parking_256", lambda: scenes.parking_256()),
]


@pytest.mark.parametrize("name,make", RENDER_CASES)
def test_render_matches_oracle(name, make):
    sc = make()
    note("render %s" % name)
    p = _planner(sc)
    p.render(_dev(sc.image), sc.vehicle)
    got = p.cspace_numpy()
    want = oracle.render(problem_of(sc), sc.image, *sc.vehicle)
    assert np.array_equal(got, want)
    p.close()


SWEEP_CASES = [(16, 8, 1.5, 1), (40, 24, 3.0, 1), (64, 64, 10.0, 1), (96, 48, 6.0, 0), (128, 128, 12.0, 1),
               (200, 72, 7.5, 1), (384, 64, 10.0, 1), (256, 256, 30.0, 1),
               # the largest sides and headings: straight lines of 1024 poses and turn
               # circles of 1024 headings (64-step sections, 16 x-major tiles per row)
               (1024, 64, 40.0, 1), (64, 1024, 12.0, 1),
               # and lengths that leave the last 64-step section short
               (1000, 16, 40.0, 1), (64, 1000, 12.0, 0)]


@pytest.mark.parametrize("N,L,R,hc", SWEEP_CASES)
def test_each_sweep_matches_oracle_on_random_values(N, L, R, hc):
    """One maneuver kernel on arbitrary pre-sweep values (random finite,
    INF, values near saturation) over a rendered cluttered volume."""
    rng = np.random.default_rng(N * 1000 + L)
    sc = scenes.random_small(int(rng.integers(1 << 30)), n=N, nt=L, R=R, half_cell=hc,
                             n_rect=max(2, N // 8)).with_(vehicle=(3, 1, 1))
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    p = _planner(sc)
    p.set_cspace(_dev(B))
    for mu in range(6):
        note("sweep %s mu=%s" % ((N, L, R, hc), oracle.NAMES[mu]))
        V = rng.integers(0, 1 << 24, size=B.shape, dtype=np.uint64).astype(np.uint32)
        V[rng.random(B.shape) < 0.3] = INF
        near = rng.random(B.shape) < 0.02
        V[near] = (INF - rng.integers(1, 1 << 16, size=int(near.sum()))).astype(np.uint32)
        p.value.copy_(_dev(V.view(np.int32)))
        p.sweep_one(mu)
        got = p.value_numpy()
        want = V.copy()
        oracle.sweep(prob, mu, B, want)
        bad = np.argwhere(got != want)
        assert bad.size == 0, (oracle.NAMES[mu], bad[:5], got[tuple(bad[0])], want[tuple(bad[0])])
    p.close()


@pytest.mark.parametrize("N,L,R", [(64, 64, 10.0), (200, 72, 7.5), (512, 40, 20.0)])
def test_straight_families_separately_match_oracle(N, L, R):
    """sweep_straight_family over both families, in either order, equals
    the oracle's straight sweep (the families hold disjoint planes)."""
    rng = np.random.default_rng(N * 7 + L)
    sc = scenes.random_small(int(rng.integers(1 << 30)), n=N, nt=L, R=R, n_rect=max(2, N // 8)).with_(
        vehicle=(3, 1, 1))
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    p = _planner(sc)
    p.set_cspace(_dev(B))
    for mu in (oracle.SF, oracle.SB):
        for order in ((0, 1), (1, 0)):
            note("straight families %s mu=%s order=%s" % ((N, L, R), oracle.NAMES[mu], order))
            V = rng.integers(0, 1 << 24, size=B.shape, dtype=np.uint64).astype(np.uint32)
            V[rng.random(B.shape) < 0.3] = INF
            p.value.copy_(_dev(V.view(np.int32)))
            for fam in order:
                p.sweep_straight_family(mu, fam)
            want = V.copy()
            oracle.sweep(prob, mu, B, want)
            assert np.array_equal(p.value_numpy(), want)
    with pytest.raises(P.NhpError) as e:
        p.sweep_straight_family(oracle.LF, 0)
    assert e.value.rc == P.EINVAL
    p.close()


PLAN_CASES = [
    ("plain_64", lambda: scenes.plain_64(), None),
    ("plain_64_s7", lambda: scenes.plain_64(7), None),
    ("small40", lambda: scenes.random_small(11, n=40, nt=24, R=3.0, n_cycles=5), 3),
    ("small96_fwd", lambda: scenes.random_small(12, n=96, nt=48, R=6.0, n_cycles=4,
                                                schedule=scenes.FORWARD_SCHEDULE), 3),
    ("clutter200", lambda: scenes.random_instance(np.random.default_rng(8), sides=(200,), thetas=(72,)), 2),
    ("clutter384", lambda: scenes.random_instance(np.random.default_rng(9), sides=(384,), thetas=(128,)), 2),
    ("parking_256", lambda: scenes.parking_256(), None),
    # short schedules: back-tracking runs one workgroup per scheduled maneuver
    ("small64_rf", lambda: scenes.random_small(16, n=64, nt=32, R=4.0, n_cycles=3, schedule=(scenes.RF,)), 6),
    ("small64_lb_sb", lambda: scenes.random_small(14, n=64, nt=40, R=4.0, n_cycles=4, schedule=(scenes.LB, scenes.SB)), 3),
]


def _oracle_plan(sc, radius):
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    V = oracle.init(prob, B, sc.start)
    oracle.cycles(prob, B, V, sc.n_cycles)
    try:
        best, score = oracle.goal_search(prob, B, V, sc.goal, radius, sc.w_xy, sc.w_t)
        steps = oracle.backtrack(prob, B, V, sc.start, best)
    except oracle.OracleError as e:
        return B, V, None, None, e.rc
    return B, V, (best, score), steps, 0


def _check_path(path, want_goal, want_steps, V):
    best, score = want_goal
    assert path.best == best and path.score == score
    assert path.value == int(V[best[2], best[1], best[0]])
    assert len(path.steps) == len(want_steps)
    for g, w in zip(path.steps, want_steps):
        assert (g.maneuver, g.steps, g.frm, g.to, g.cost) == (w.maneuver, w.steps, w.frm, w.to, w.cost)


@pytest.mark.parametrize("name,make,radius", PLAN_CASES)
def test_full_plan_matches_oracle(name, make, radius):
    sc = make()
    radius = sc.goal_radius if radius is None else radius
    note("plan %s %dx%dx%d N=%d" % (name, sc.nx, sc.nx, sc.nt, sc.n_cycles))
    B, V, goal, steps, rc = _oracle_plan(sc, radius)
    p = _planner(sc)
    p.render(_dev(sc.image), sc.vehicle)
    p.sweep(sc.start, sc.n_cycles)
    assert np.array_equal(p.cspace_numpy(), B)
    got = p.value_numpy()
    assert np.array_equal(got, V)
    if rc:
        with pytest.raises(P.NhpError) as e:
            p.extract(sc.goal, radius, sc.w_xy, sc.w_t)
        assert e.value.rc == rc
    else:
        path = p.extract(sc.goal, radius, sc.w_xy, sc.w_t)
        _check_path(path, goal, steps, V)
    p.close()


def test_resume_and_determinism():
    sc = scenes.random_small(21, n=64, nt=64, R=8.0, n_cycles=4)
    p = _planner(sc)
    p.render(_dev(sc.image), sc.vehicle)
    p.sweep(sc.start, 4)
    a = p.value_numpy()
    p.sweep(sc.start, 1)
    p.resume(3)
    b = p.value_numpy()
    p.sweep(sc.start, 4)
    c = p.value_numpy()
    assert np.array_equal(a, b) and np.array_equal(a, c)
    p.close()


def test_error_paths():
    sc = scenes.plain_64()
    p = _planner(sc)
    with pytest.raises(P.NhpError) as e:
        p.sweep(sc.start, 1)
    assert e.value.rc == P.ESTATE
    with pytest.raises(P.NhpError) as e:
        p.extract(sc.goal)
    assert e.value.rc == P.ESTATE
    p.render(_dev(sc.image), sc.vehicle)
    with pytest.raises(P.NhpError) as e:
        p.sweep((0, 5, 0), 1)  # the wall
    assert e.value.rc == P.ESTART
    with pytest.raises(P.NhpError) as e:
        p.sweep((64, 5, 0), 1)
    assert e.value.rc == P.EINVAL
    p.sweep(sc.start, 0)  # only the start is reached
    with pytest.raises(P.NhpError) as e:
        p.extract(sc.goal, 0)
    assert e.value.rc == P.EUNREACH
    p.sweep(sc.start, sc.n_cycles)
    path = p.extract(sc.goal, 2)
    if len(path.steps) > 1:
        with pytest.raises(P.NhpError) as e:
            p.extract(sc.goal, 2, cap=1)
        assert e.value.rc == P.ECAP
    with pytest.raises(P.NhpError) as e:
        p.extract(sc.goal, 40)
    assert e.value.rc == P.EINVAL
    p.close()


def test_maze_512_full_size():
    """The 512^3, N = 20 maze at full size, in the launch configuration the
    benchmark times: obstacle volume, value volume after all 120 sweeps and
    the extracted plan, bit for bit against the oracle."""
    sc = scenes.maze_512()
    note("maze_512: GPU")
    p = _planner(sc)
    p.render(_dev(sc.image), sc.vehicle)
    p.sweep(sc.start, sc.n_cycles)
    got_B, got_V = p.cspace_numpy(), p.value_numpy()
    path = None
    try:
        path = p.extract(sc.goal, sc.goal_radius, sc.w_xy, sc.w_t)
    except P.NhpError as e:
        path = e
    p.close()
    note("maze_512: oracle")
    t = time.time()
    B, V, goal, steps, rc = _oracle_plan(sc, sc.goal_radius)
    note("maze_512: oracle %.1f s" % (time.time() - t))
    assert np.array_equal(got_B, B)
    assert np.array_equal(got_V, V)
    if rc:
        assert isinstance(path, P.NhpError) and path.rc == rc
    else:
        _check_path(path, goal, steps, V)


def test_graph_replays_match_eager_launches():
    """sweep_n_turns replays a captured cycle graph; every replay, with eager
    work and synchronisations between replays, matches cycles launched one
    kernel at a time through sweep_one."""
    sc = scenes.random_small(31, n=96, nt=48, R=6.0, n_cycles=3)
    p = _planner(sc)
    p.render(_dev(sc.image), sc.vehicle)
    for rep in range(4):
        p.sweep(sc.start, rep + 1)          # graph replays
        graph = p.value_numpy()
        p.sweep(sc.start, 0)                # eager: init only, then one kernel per sweep
        for _ in range(rep + 1):
            for mu in sc.schedule:
                p.sweep_one(mu)
        eager = p.value_numpy()
        torch.cuda.synchronize()
        assert np.array_equal(graph, eager), rep
    p.close()


@pytest.mark.parametrize("N,L", [(128, 128), (96, 72)])
def test_every_section_size_matches_oracle(N, L):
    """Every section size the tuner may pick gives the oracle's values."""
    rng = np.random.default_rng(N + L)
    sc = scenes.random_small(int(rng.integers(1 << 30)), n=N, nt=L, R=6.0, n_rect=N // 8).with_(vehicle=(3, 1, 1))
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    V0 = rng.integers(0, 1 << 22, size=B.shape, dtype=np.uint64).astype(np.uint32)
    V0[rng.random(B.shape) < 0.4] = INF
    try:
        for steps in (8, 16, 32, 64):
            if (L + steps - 1) // steps > 16 and (N + steps - 1) // steps > 16:
                continue
            for length in (N, L):
                if (length + steps - 1) // steps <= 16:
                    P.set_section_steps(length, steps)
            p = _planner(sc)
            p.set_cspace(_dev(B))
            for mu in range(6):
                note("section %d %s mu=%s" % (steps, (N, L), oracle.NAMES[mu]))
                p.value.copy_(_dev(V0.view(np.int32)))
                p.sweep_one(mu)
                want = V0.copy()
                oracle.sweep(prob, mu, B, want)
                assert np.array_equal(p.value_numpy(), want), (steps, mu)
            p.close()
    finally:
        P.set_section_steps(N, 0)
        P.set_section_steps(L, 0)
        P.apply_tuning()


def _farthest_reached(B, V):
    """The free, reached pose of largest value (first in memory order on a
    tie): a goal whose plan walks back across most of the volume."""
    flat = V.reshape(-1)
    free = (B.reshape(-1) != 255) & (flat != INF)
    vmax = flat[free].max()
    q = int(np.flatnonzero(free & (flat == vmax))[0])
    L, N, _ = V.shape
    return (q % N, (q // N) % N, q // (N * N))


def _plan_to_farthest(sc):
    """Oracle volumes of the scene, then the farthest reached pose as goal
    (radius 0) with its goal search and back-tracking."""
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    V = oracle.init(prob, B, sc.start)
    oracle.cycles(prob, B, V, sc.n_cycles)
    goal = _farthest_reached(B, V)
    best, score = oracle.goal_search(prob, B, V, goal, 0, sc.w_xy, sc.w_t)
    steps = oracle.backtrack(prob, B, V, sc.start, best)
    return B, V, goal, (best, score), steps


# Curves longer than 512 poses (straight lines of 1024 cells, circles of
# 1024 headings) through the whole single-plan path, so back-tracking runs
# its 1024-thread workgroups; and the largest grid of the batched workload.
LONG_CASES = [
    ("wide1024x64", lambda: scenes.random_instance(np.random.default_rng(12), sides=(1024,), thetas=(64,),
                                                   n_range=(2, 2), name="wide1024x64")),
    ("tall64x1024", lambda: scenes.random_instance(np.random.default_rng(13), sides=(64,), thetas=(1024,),
                                                   n_range=(2, 2), len_range=(4, 6), name="tall64x1024")),
    ("clutter384x256", lambda: scenes.random_instance(np.random.default_rng(10), sides=(384,), thetas=(256,),
                                                      name="clutter384x256")),
]


@pytest.mark.parametrize("name,make", LONG_CASES)
def test_long_curves_full_plan_matches_oracle(name, make):
    sc = make()
    note("plan %s %dx%dx%d N=%d" % (name, sc.nx, sc.nx, sc.nt, sc.n_cycles))
    B, V, goal, want_goal, steps = _plan_to_farthest(sc)
    assert len(steps) >= 2, "the farthest reached pose needs a multi-step plan"
    p = _planner(sc)
    p.render(_dev(sc.image), sc.vehicle)
    p.sweep(sc.start, sc.n_cycles)
    assert np.array_equal(p.cspace_numpy(), B)
    assert np.array_equal(p.value_numpy(), V)
    path = p.extract(goal, 0, sc.w_xy, sc.w_t)
    _check_path(path, want_goal, steps, V)
    p.close()


def test_largest_serving_request_full_size():
    """The largest request of the serving workload, 1024 x 1024 cells x 512
    headings (a 2 GiB value volume, 1024-pose straight lines and 512-heading
    circles), N = 4 cycles, in the launch configuration the benchmark uses:
    obstacle volume, value volume and the plan to the farthest reached pose,
    bit for bit against the oracle."""
    sc = scenes.random_instance(np.random.default_rng(1306), sides=(1024,), thetas=(512,), n_range=(4, 4),
                                occ=(0.15, 0.15), name="request1024")
    note("request1024: GPU")
    p = _planner(sc)
    p.render(_dev(sc.image), sc.vehicle)
    p.sweep(sc.start, sc.n_cycles)
    got_B, got_V = p.cspace_numpy(), p.value_numpy()
    note("request1024: oracle")
    t = time.time()
    B, V, goal, want_goal, steps = _plan_to_farthest(sc)
    note("request1024: oracle %.1f s, plan of %d steps" % (time.time() - t, len(steps)))
    assert np.array_equal(got_B, B)
    del got_B, B
    assert np.array_equal(got_V, V)
    del got_V
    path = p.extract(goal, 0, sc.w_xy, sc.w_t)
    p.close()
    _check_path(path, want_goal, steps, V)
