"""Host logic of the pass grouping (no GPU): which consecutive maneuver
sweeps share one pass over the value volume.  Two turns share a pass when
they run over the same circles (left: LF, LB; right: RF, RB, eqs. 25-28) in
opposite directions; the grouping must keep the sweep order of the schedule
(Insert 1 applies the maneuvers one after another)."""
import itertools

import pytest

from paper_2306_01301_amd import planner as P

LF, SF, RB, RF, SB, LB = range(6)
LEFT, RIGHT = {LF, LB}, {RF, RB}


def fusable(a, b):
    return a != b and ({a, b} <= LEFT or {a, b} <= RIGHT)


def _check(schedule, first, count, pairs=True):
    passes = P.schedule_passes(schedule, first, count, pairs)
    seq = [schedule[k % len(schedule)] for k in range(first, first + count)]
    flat = [m for a, b in passes for m in ((a,) if b < 0 else (a, b))]
    assert flat == seq  # same sweeps, same order
    k = 0
    for a, b in passes:
        if b >= 0:
            assert pairs and fusable(a, b)
            k += 2
        else:
            # greedy: a single is never followed by a partner it could take
            if pairs and k + 1 < len(seq):
                assert not fusable(seq[k], seq[k + 1])
            k += 1
    return passes


def test_default_schedule():
    sched = (LF, SF, RB, RF, SB, LB)
    passes = _check(sched, 0, 6 * 20)
    # LF alone, then per cycle SF, RB+RF, SB, LB+LF, and LB alone at the end
    assert passes[:5] == [(LF, -1), (SF, -1), (RB, RF), (SB, -1), (LB, LF)]
    assert passes[-1] == (LB, -1)
    assert len(passes) == 1 + 19 * 4 + 4
    assert _check(sched, 0, 120, pairs=False) == [(m, -1) for m in sched] * 20


def test_every_short_schedule():
    for n in (1, 2, 3):
        for sched in itertools.product(range(6), repeat=n):
            for first in range(0, 2 * n):
                for count in range(0, 3 * n + 1):
                    _check(sched, first, count)


def test_errors():
    with pytest.raises(P.NhpError):
        P.schedule_passes((0, 7), 0, 4)
    with pytest.raises(P.NhpError):
        P.schedule_passes((), 0, 4)
