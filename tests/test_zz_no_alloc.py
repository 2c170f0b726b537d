"""extract_path_noalloc (the extract entry point that allocates nothing)
against extract_path on the same plans, through the C ABI: two calls in a
row, the second on a smaller plan, and the step-buffer and error paths."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2306_01301_amd import planner, scenes

pytestmark = pytest.mark.gpu


def _path_tuple(path):
    return (path.best, path.value, path.score,
            [(s.maneuver, s.steps, s.frm, s.to, s.cost) for s in path.steps])


def _swept(sc):
    p = planner.planner_for(sc)
    img = torch.from_numpy(np.ascontiguousarray(sc.image)).cuda()
    p.render(img, sc.vehicle)
    p.sweep(sc.start, sc.n_cycles)
    return p


def test_noalloc_extract_equals_extract_path_larger_then_smaller():
    big, small = scenes.parking_256(), scenes.plain_64()
    want, got = [], []
    for sc in (big, small):  # the second call is on the smaller plan
        print("no-alloc extract:", sc.name, sc.nx, sc.nt, flush=True)
        p = _swept(sc)
        r = sc.goal_radius
        got.append(_path_tuple(p.extract_noalloc(sc.goal, r, sc.w_xy, sc.w_t)))
        want.append(_path_tuple(p.extract(sc.goal, r, sc.w_xy, sc.w_t)))
        # and once more after extract_path, on the same plan
        assert _path_tuple(p.extract_noalloc(sc.goal, r, sc.w_xy, sc.w_t)) == want[-1]
        p.close()
    assert len(want[0][3]) > 1 and len(want[1][3]) > 1
    assert got == want


def test_noalloc_extract_step_buffer_and_errors():
    sc = scenes.plain_64()
    p = _swept(sc)
    want = p.extract(sc.goal, sc.goal_radius, sc.w_xy, sc.w_t)
    n = len(want.steps)
    assert n >= 2
    # a buffer of exactly the plan's length
    exact = (planner.NhpStep * n)()
    assert _path_tuple(p.extract_noalloc(sc.goal, sc.goal_radius, sc.w_xy, sc.w_t, steps=exact)) == _path_tuple(want)
    # one step short: NHP_ECAP with the needed length reported
    short = (planner.NhpStep * (n - 1))()
    nn = ctypes.c_uint32()
    gi, gj, gt = sc.goal
    rc = planner.lib().extract_path_noalloc(p._plan, gi, gj, gt, sc.goal_radius, sc.w_xy, sc.w_t, short, n - 1,
                                            ctypes.byref(nn), None, None, None)
    assert rc == planner.ECAP and nn.value == n
    # a goal outside the grid
    rc = planner.lib().extract_path_noalloc(p._plan, sc.nx, 0, 0, 0, 0, 0, short, n - 1, ctypes.byref(nn), None,
                                            None, None)
    assert rc == planner.EINVAL
    p.close()
