"""GPU parity of the batched entry points (batch_render / batch_sweep /
batch_step / batch_extract): many plans of uneven sizes in shared launches
give, plan by plan, exactly what the oracle gives, and a plan's result is
the same alone and in a mix where other plans join and leave at other ticks
(continuous batching)."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2306_01301_amd import planner as P
from paper_2306_01301_amd import scenes
from tests.common import problem_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    oracle.set_threads(min(16, os.cpu_count() or 1))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _mixed_scenes():
    rng = np.random.default_rng(4242)
    out = [
        scenes.plain_64(),
        scenes.random_small(101, n=40, nt=24, R=3.0, n_cycles=3),
        scenes.random_small(102, n=96, nt=48, R=6.0, n_cycles=2, schedule=scenes.FORWARD_SCHEDULE),
        scenes.random_small(103, n=48, nt=64, R=5.0, n_cycles=5, half_cell=0),
        scenes.random_instance(rng, sides=(128,), thetas=(128,), n_range=(3, 3)),
        scenes.random_instance(rng, sides=(200,), thetas=(72,), n_range=(2, 2)),
        scenes.random_instance(rng, sides=(256,), thetas=(128,), n_range=(1, 1)),
        scenes.random_small(104, n=16, nt=8, R=1.5, n_cycles=4),
    ]
    return out


def _oracle(sc, radius):
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    V = oracle.init(prob, B, sc.start)
    oracle.cycles(prob, B, V, sc.n_cycles)
    try:
        best, score = oracle.goal_search(prob, B, V, sc.goal, radius, sc.w_xy, sc.w_t)
        steps = oracle.backtrack(prob, B, V, sc.start, best)
        return B, V, (best, score, steps)
    except oracle.OracleError as e:
        return B, V, e.rc


def test_batch_matches_oracle():
    scs = _mixed_scenes()
    planners = [P.planner_for(sc) for sc in scs]
    batch = P.Batch(len(scs))
    images = [_dev(sc.image) for sc in scs]
    batch.render(planners, images, [sc.vehicle for sc in scs])
    batch.sweep(planners, [sc.start for sc in scs], [sc.n_cycles for sc in scs])
    radius = [3] * len(scs)
    paths = batch.extract(planners, [sc.goal for sc in scs], radius, [sc.w_xy for sc in scs],
                          [sc.w_t for sc in scs])
    for k, sc in enumerate(scs):
        print("batch plan %d: %s %dx%dx%d N=%d" % (k, sc.name, sc.nx, sc.nx, sc.nt, sc.n_cycles), flush=True)
        B, V, want = _oracle(sc, radius[k])
        assert np.array_equal(planners[k].cspace_numpy(), B), k
        assert np.array_equal(planners[k].value_numpy(), V), k
        if isinstance(want, int):
            assert paths[k] == want, k
        else:
            best, score, steps = want
            got = paths[k]
            assert not isinstance(got, int), (k, got)
            assert got.best == best and got.score == score
            assert [(s.maneuver, s.steps, s.frm, s.to, s.cost) for s in got.steps] == \
                   [(s.maneuver, s.steps, s.frm, s.to, s.cost) for s in steps]
    batch.close()
    for p in planners:
        p.close()


def test_same_alone_and_in_a_continuous_batch():
    """Plans join at different ticks and leave when done; every tick advances
    every live plan by one sweep in shared launches.  Each final value volume
    equals the same plan run alone through sweep_n_turns."""
    scs = _mixed_scenes()
    join = [0, 3, 1, 7, 2, 11, 5, 4]
    planners = [P.planner_for(sc) for sc in scs]
    batch = P.Batch(len(scs))
    for p, sc in zip(planners, scs):
        p.render(_dev(sc.image), sc.vehicle)
    total = [sc.n_cycles * len(sc.schedule) for sc in scs]
    done = [0] * len(scs)
    tick = 0
    while any(done[k] < total[k] for k in range(len(scs))):
        newcomers = [k for k in range(len(scs)) if join[k] == tick]
        if newcomers:
            batch.init([planners[k] for k in newcomers], [scs[k].start for k in newcomers])
        live = [k for k in range(len(scs)) if join[k] <= tick and done[k] < total[k]]
        if live:
            batch.step([planners[k] for k in live], [done[k] for k in live])
            for k in live:
                done[k] += 1
        tick += 1
    mixed = [p.value_numpy() for p in planners]
    batch.close()
    for k, (p, sc) in enumerate(zip(planners, scs)):
        p.sweep(sc.start, sc.n_cycles)
        assert np.array_equal(p.value_numpy(), mixed[k]), k
        p.close()


def test_batch_errors():
    sc = scenes.plain_64()
    a, b = P.planner_for(sc), P.planner_for(sc)
    batch = P.Batch(2)
    with pytest.raises(P.NhpError) as e:
        batch.init([a], [sc.start])
    assert e.value.rc == P.ESTATE
    batch.render([a, b], [_dev(sc.image)] * 2, [sc.vehicle] * 2)
    with pytest.raises(P.NhpError) as e:
        batch.step([a], [0])
    assert e.value.rc == P.ESTATE
    with pytest.raises(P.NhpError) as e:
        batch.init([a, a], [sc.start, sc.start])
    assert e.value.rc == P.EINVAL
    with pytest.raises(P.NhpError) as e:
        batch.init([a, b], [sc.start, (0, 3, 0)])
    assert e.value.rc == P.ESTART
    c = P.planner_for(sc)
    with pytest.raises(P.NhpError) as e:
        batch.init([a, b, c], [sc.start] * 3)  # over capacity
    assert e.value.rc == P.EINVAL
    batch.close()
    for p in (a, b, c):
        p.close()


def _config4_scenes():
    """The grid shapes of the batched workload (384 and 256 sides with 256
    and 128 headings, 128^2 x 128), with the workload's N, clutter and
    vehicles, plus circles of 1024 headings (batched back-tracking over
    curves longer than 512 poses)."""
    rng = np.random.default_rng(4343)
    shapes = [(384, 256), (384, 128), (256, 256), (128, 128)]
    out = [scenes.random_instance(rng, sides=(n,), thetas=(t,), name="c4_%dx%d" % (n, t)) for n, t in shapes]
    out.append(scenes.random_instance(rng, sides=(64,), thetas=(1024,), n_range=(2, 2), len_range=(4, 6),
                                      name="tall64x1024"))
    return out


def _farthest_goal(sc):
    """Oracle volumes and the free reached pose of largest value (first in
    memory order) as the goal, so every plan back-tracks a long way."""
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    V = oracle.init(prob, B, sc.start)
    oracle.cycles(prob, B, V, sc.n_cycles)
    flat = V.reshape(-1)
    free = (B.reshape(-1) != 255) & (flat != 0xFFFFFFFF)
    q = int(np.flatnonzero(free & (flat == flat[free].max()))[0])
    N = sc.nx
    goal = (q % N, (q // N) % N, q // (N * N))
    best, score = oracle.goal_search(prob, B, V, goal, 0, sc.w_xy, sc.w_t)
    return B, V, goal, (best, score, oracle.backtrack(prob, B, V, sc.start, best))


def test_batch_of_config4_shapes_matches_oracle():
    """Plans of the batched workload's largest shapes in shared launches:
    obstacle volume, value volume and plan of each, bit for bit."""
    scs = _config4_scenes()
    want = []
    for sc in scs:
        print("oracle %s %dx%dx%d N=%d" % (sc.name, sc.nx, sc.nx, sc.nt, sc.n_cycles), flush=True)
        want.append(_farthest_goal(sc))
    planners = [P.planner_for(sc) for sc in scs]
    batch = P.Batch(len(scs))
    batch.render(planners, [_dev(sc.image) for sc in scs], [sc.vehicle for sc in scs])
    batch.sweep(planners, [sc.start for sc in scs], [sc.n_cycles for sc in scs])
    paths = batch.extract(planners, [w[2] for w in want], [0] * len(scs), [sc.w_xy for sc in scs],
                          [sc.w_t for sc in scs], cap=1024)
    for k, sc in enumerate(scs):
        B, V, goal, (best, score, steps) = want[k]
        assert np.array_equal(planners[k].cspace_numpy(), B), sc.name
        assert np.array_equal(planners[k].value_numpy(), V), sc.name
        got = paths[k]
        assert not isinstance(got, int), (sc.name, got)
        assert len(steps) >= 2, sc.name
        assert got.best == best and got.score == score, sc.name
        assert [(s.maneuver, s.steps, s.frm, s.to, s.cost) for s in got.steps] == \
               [(s.maneuver, s.steps, s.frm, s.to, s.cost) for s in steps], sc.name
    batch.close()
    for p in planners:
        p.close()


def test_batch_cycle_graph_replays_match_oracle():
    """batch_sweep replays repeated cycles from captured graphs (within a
    call from the third cycle on, and whole calls on the same plans): the
    same plans swept again with new starts, with other GPU work and
    synchronisations between the calls, match the oracle every time."""
    rng = np.random.default_rng(4343)
    scs = [scenes.random_small(201, n=64, nt=64, R=6.0, n_cycles=6),
           scenes.random_small(202, n=48, nt=40, R=4.0, n_cycles=5),
           scenes.random_instance(rng, sides=(128,), thetas=(128,), n_range=(6, 6))]
    planners = [P.planner_for(sc) for sc in scs]
    batch = P.Batch(len(scs))
    batch.render(planners, [_dev(sc.image) for sc in scs], [sc.vehicle for sc in scs])
    for rep in range(4):
        starts = []
        for sc in scs:  # a new collision-free start per repetition (the first: the scene's own)
            prob = problem_of(sc)
            B = oracle.render(prob, sc.image, *sc.vehicle)
            if rep == 0:
                starts.append(tuple(sc.start))
                continue
            free = np.argwhere(B != 255)
            t, j, i = free[rng.integers(len(free))]
            starts.append((int(i), int(j), int(t)))
        print("batch graph replay %d starts %s" % (rep, starts), flush=True)
        batch.sweep(planners, starts, [sc.n_cycles for sc in scs])
        torch.zeros(1 << 20, device="cuda").add_(1.0)  # other work between the calls
        torch.cuda.synchronize()
        for k, sc in enumerate(scs):
            prob = problem_of(sc)
            B = oracle.render(prob, sc.image, *sc.vehicle)
            V = oracle.init(prob, B, starts[k])
            oracle.cycles(prob, B, V, sc.n_cycles)
            assert np.array_equal(planners[k].value_numpy(), V), (rep, k)
    batch.close()
    for p in planners:
        p.close()
