"""The server's tick policy (host logic, no GPU): which plans advance and by
how many sweeps."""
from types import SimpleNamespace

from paper_2306_01301_amd import planner as P
from paper_2306_01301_amd import serving


def _live(k, n, nt, cycles, arrival, done=0):
    sc = SimpleNamespace(n_poses=n * n * nt, schedule=P.DEFAULT_SCHEDULE)
    return serving._Live(k, sc, None, None, 6 * cycles, arrival, done=done)


def test_shortest_remaining_work_first_until_the_launches_fill():
    plans = [_live(0, 384, 256, 12, 0.0), _live(1, 128, 128, 4, 0.0), _live(2, 256, 128, 8, 0.0),
             _live(3, 128, 128, 4, 0.0, done=24)]  # plan 3 has all its sweeps enqueued
    picked = serving.tick_plan(plans, 0.0, fill_poses=3 << 20, tick_poses=1 << 20, aging=0.0)
    # plan 1 (2 M poses) then plan 2 (8 M poses) reach the fill target; plan 0 waits
    assert [l.k for l, _ in picked] == [1, 2]
    # whole passes: plan 1 gets one pass (its first, LF), plan 2 one pass
    assert [n for _, n in picked] == [1, 1]
    everything = serving.tick_plan(plans, 0.0, fill_poses=1 << 40, tick_poses=1 << 40, aging=0.0)
    assert sorted(l.k for l, _ in everything) == [0, 1, 2]
    assert all(l.done + n == l.total for l, n in everything)  # a large tick finishes every plan


def test_passes_end_on_pass_boundaries():
    (l, n), = serving.tick_plan([_live(0, 64, 64, 3, 0.0, done=1)], 0.0, fill_poses=1, tick_poses=3 * 64 * 64 * 64)
    # sweeps 1.. of LF SF RB RF SB LB: SF, then RB+RF fused (2 sweeps), then SB: three passes = 4 sweeps
    assert n == 4


def test_aging_moves_an_old_large_request_ahead():
    big, small = _live(0, 512, 512, 20, 0.0), _live(1, 128, 128, 4, 5.0)
    first = serving.tick_plan([big, small], 5.0, fill_poses=1, aging=0.0)[0][0]
    assert first.k == 1
    first = serving.tick_plan([big, small], 5.0, fill_poses=1, aging=1.0)[0][0]
    assert first.k == 0  # 5 s in the system outweigh its ~0.3 s of expected work
