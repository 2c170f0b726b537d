"""GPU parity of maneuver-count reachability (App. C): obstacle bits, every
level volume, goal search and back-tracking through the C ABI against the
oracle, bit for bit.  Sizes cover rows of one word, word counts that are not
powers of two (idle lanes), curve lengths that are not a multiple of the
section size, every schedule shape, every turn section length (4 to 32
steps) and the full 128 x 128 x 512, N = 8 workload."""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2306_01301_amd import planner as P
from paper_2306_01301_amd import scenes
from tests.common import problem_of

pytestmark = pytest.mark.gpu

HARD = 255
LF, SF, RB, RF, SB, LB = range(6)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    oracle.set_threads(min(16, os.cpu_count() or 1))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _words_to_bits(t, shape):
    w = t.cpu().numpy().view(np.uint32)
    return np.unpackbits(w.view(np.uint8), bitorder="little").astype(bool).reshape(shape)


def _levels(reach, n_cycles, shape):
    torch.cuda.synchronize()
    return P.bits_to_levels([reach.level_words(m).cpu().numpy().view(np.uint32) for m in range(n_cycles + 1)], shape)


CASES = [
    # seed, n, nt, R, schedule, cycles, vehicle
    (1, 32, 16, 2.5, scenes.DEFAULT_SCHEDULE, 4, (1, 0, 0)),
    (2, 64, 64, 6.0, scenes.DEFAULT_SCHEDULE, 5, (3, 1, 1)),
    (3, 96, 72, 6.0, scenes.FORWARD_SCHEDULE, 4, (2, 1, 1)),
    (4, 160, 40, 8.0, (LB, SB, RB), 3, (3, 1, 1)),
    (5, 128, 256, 12.0, (LF, SF, RF, LB), 3, (4, 1, 2)),
    (6, 64, 512, 10.0, (RF,), 2, (2, 1, 1)),
    # turn sections of 16 and 32 steps (the section length grows with the
    # words per row so that a workgroup holds a whole row of curves)
    (7, 256, 512, 10.0, scenes.DEFAULT_SCHEDULE, 2, (3, 1, 1)),
    (8, 512, 512, 10.0, (LB, SF, RF), 1, (3, 1, 1)),
]


@pytest.mark.parametrize("seed,n,nt,R,sched,ncyc,veh", CASES)
def test_reach_matches_oracle(seed, n, nt, R, sched, ncyc, veh):
    sc = scenes.random_small(seed, n=n, nt=nt, R=R, schedule=sched, n_rect=max(3, n // 8)).with_(vehicle=veh)
    prob = problem_of(sc)
    note("reach %s" % ((seed, n, nt, R, [oracle.NAMES[m] for m in sched], ncyc),))
    B = oracle.render(prob, sc.image, *veh)
    pl = P.planner_for(sc)
    rc = P.Reach(pl, ncyc)
    rc.render(_dev(sc.image), veh)
    torch.cuda.synchronize()
    assert np.array_equal(_words_to_bits(rc.hard_words(), B.shape), B == HARD)
    start = sc.start
    if B[start[2], start[1], start[0]] == HARD:
        pytest.skip("start in collision")
    rc.sweep(start, ncyc)
    want = oracle.reach(prob, B, start, ncyc)
    got = _levels(rc, ncyc, B.shape)
    bad = np.argwhere(got != want)
    assert bad.size == 0, (bad[:5], got[tuple(bad[0])], want[tuple(bad[0])])
    for radius in (0, 3):
        try:
            best, lv = oracle.reach_goal(prob, want, sc.goal, radius)
        except oracle.OracleError:
            with pytest.raises(P.NhpError) as e:
                rc.extract(sc.goal, radius)
            assert e.value.rc == P.EUNREACH
            continue
        steps = oracle.reach_backtrack(prob, B, want, best)
        path = rc.extract(sc.goal, radius)
        assert path.best == best and path.level == lv
        assert [(s.maneuver, s.steps, s.frm, s.to, s.cost) for s in path.steps] == \
               [(s.maneuver, s.steps, s.frm, s.to, s.cost) for s in steps]
    rc.close()
    pl.close()


def test_reach_from_code_volume():
    """reach_set_cspace takes the hard bits of a code volume; the levels then
    follow exactly as from rendering."""
    sc = scenes.random_small(21, n=64, nt=48, R=5.0, n_rect=8).with_(vehicle=(2, 1, 1))
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    pl = P.planner_for(sc)
    rc = P.Reach(pl, 4)
    rc.set_cspace(_dev(B))
    torch.cuda.synchronize()
    assert np.array_equal(_words_to_bits(rc.hard_words(), B.shape), B == HARD)
    rc.sweep(sc.start, 4)
    assert np.array_equal(_levels(rc, 4, B.shape), oracle.reach(prob, B, sc.start, 4))
    rc.close()
    pl.close()


def test_reach_128_full_size():
    sc = scenes.reach_128()
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    pl = P.planner_for(sc)
    rc = P.Reach(pl, sc.n_cycles)
    rc.render(_dev(sc.image), sc.vehicle)
    rc.sweep(sc.start, sc.n_cycles)
    torch.cuda.synchronize()
    assert np.array_equal(_words_to_bits(rc.hard_words(), B.shape), B == HARD)
    want = oracle.reach(prob, B, sc.start, sc.n_cycles)
    assert np.array_equal(_levels(rc, sc.n_cycles, B.shape), want)
    best, lv = oracle.reach_goal(prob, want, sc.goal, 0)
    steps = oracle.reach_backtrack(prob, B, want, best)
    path = rc.extract(sc.goal, 0)
    assert path.best == best and path.level == lv == len(steps)
    assert [(s.maneuver, s.steps, s.frm, s.to) for s in path.steps] == [(s.maneuver, s.steps, s.frm, s.to) for s in steps]
    # the cycles replay from a captured graph: again from another start, with
    # eager work and a synchronisation between the replays, then the first again
    other = (sc.goal[0], sc.goal[1], sc.goal[2])
    for start in (other, sc.start, other):
        if B[start[2], start[1], start[0]] == HARD:
            continue
        rc.sweep(start, sc.n_cycles)
        torch.cuda.synchronize()
        assert np.array_equal(_levels(rc, sc.n_cycles, B.shape), oracle.reach(prob, B, start, sc.n_cycles))
        rc.sweep(start, 2)  # a two-cycle sweep in between (launched directly: a count used once is not captured)
        torch.cuda.synchronize()
        assert np.array_equal(_levels(rc, 2, B.shape), oracle.reach(prob, B, start, 2))
    rc.close()
    pl.close()


def test_reach_errors():
    sc = scenes.random_small(31, n=40, nt=16, R=3.0)
    pl = P.planner_for(sc)
    with pytest.raises(P.NhpError) as e:
        P.Reach(pl, 2)  # 40 is not a multiple of 32
    assert e.value.rc == P.EINVAL
    pl.close()
    sc = scenes.random_small(32, n=64, nt=16, R=3.0)
    pl = P.planner_for(sc)
    rc = P.Reach(pl, 2)
    with pytest.raises(P.NhpError) as e:
        rc.sweep(sc.start, 1)
    assert e.value.rc == P.ESTATE
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    rc.set_cspace(_dev(B))
    with pytest.raises(P.NhpError) as e:
        rc.extract(sc.goal)
    assert e.value.rc == P.ESTATE
    with pytest.raises(P.NhpError) as e:
        rc.sweep((0, 5, 0), 1)  # the wall column is hard
    assert e.value.rc == P.ESTART
    with pytest.raises(P.NhpError) as e:
        rc.sweep(sc.start, 3)  # more cycles than the state keeps
    assert e.value.rc == P.EINVAL
    rc.close()
    pl.close()
