"""Launch-shape knobs (nhp_set_knob) change speed only: every maneuver
kernel under every tested setting gives the oracle's result, bit for bit."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2306_01301_amd import planner as P
from paper_2306_01301_amd import scenes
from tests.common import problem_of

pytestmark = pytest.mark.gpu

INF = 0xFFFFFFFF
SETTINGS = [
    {},
    {"row_wg_per_cu": 1, "xmajor_wg_per_cu": 4, "tile_order": 2, "xmajor_buffers": 1},
    {"row_wg_per_cu": 2, "xmajor_wg_per_cu": 16, "tile_order": 1, "xmajor_buffers": 2},
    {"xmajor_buffers": 1},
    # one x-major workgroup per CU: band tiles walk several tiles each (the
    # dirty-row flags and their chunk parity carry across tiles)
    {"xmajor_wg_per_cu": 1},
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    oracle.set_threads(min(16, os.cpu_count() or 1))
    yield
    for k in P.KNOBS.values():
        P.set_knob(k, 0)
    P.apply_tuning()


@pytest.mark.parametrize("N,L,R", [(200, 72, 7.5), (512, 40, 20.0), (64, 256, 10.0), (512, 128, 16.0)])
@pytest.mark.parametrize("setting", range(len(SETTINGS)))
def test_every_knob_setting_matches_oracle(N, L, R, setting):
    for name in P.KNOBS:
        P.set_knob(P.KNOBS[name], SETTINGS[setting].get(name, 0))
    rng = np.random.default_rng(N + L + setting)
    sc = scenes.random_small(int(rng.integers(1 << 30)), n=N, nt=L, R=R, n_rect=max(2, N // 8)).with_(
        vehicle=(3, 1, 1))
    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    p = P.planner_for(sc)
    p.set_cspace(torch.from_numpy(B).cuda())
    for first, second in ((P.SF, -1), (P.SB, -1), (P.LF, -1), (P.RB, P.RF)):
        print("knobs %s %s pass %s" % (SETTINGS[setting], (N, L, R), (first, second)), flush=True)
        V = rng.integers(0, 1 << 24, size=B.shape, dtype=np.uint64).astype(np.uint32)
        V[rng.random(B.shape) < 0.3] = INF
        p.value.copy_(torch.from_numpy(V.view(np.int32)).cuda())
        p.sweep_pass(first, second)
        want = V.copy()
        oracle.sweep(prob, first, B, want)
        if second >= 0:
            oracle.sweep(prob, second, B, want)
        assert np.array_equal(p.value_numpy(), want)
    p.close()
