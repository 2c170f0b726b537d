"""Serving on the GPU: the continuous-batching server, one plan per launch
and one batch give every request the same value volume and the same plan;
requests that arrive while others run are admitted and overlap."""
import numpy as np
import pytest
import torch

from paper_2306_01301_amd import planner as P
from paper_2306_01301_amd import scenes, serving

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


def _requests(count):
    rng = np.random.default_rng(77)
    return [scenes.random_instance(rng, sides=(64, 128, 192), thetas=(64, 128), n_range=(2, 5),
                                   name="r%02d" % k) for k in range(count)]


def _key(r):
    p = r.path
    steps = None if p is None else [(s.maneuver, s.steps, s.frm, s.to, s.cost) for s in p.steps]
    return (r.status, r.value_digest, None if p is None else (p.best, p.value, p.score), steps)


def test_alone_in_a_batch_and_served_agree():
    reqs = _requests(12)
    single = serving.run_single(reqs, digests=True)
    batched = serving.run_batched(reqs, digests=True)
    arrivals = scenes.poisson_arrivals(5, 400.0, len(reqs))
    budget = 3 * max(serving.footprint_bytes(sc) for sc in reqs)  # forces queueing
    srv = serving.Server(budget, max_live=8, digests=True)
    served = srv.run(reqs, arrivals)
    srv.close()
    for a, b, c in zip(single, batched, served):
        assert _key(a) == _key(b) == _key(c), a.name
    # requests overlapped: one was admitted while an earlier one was still running
    assert any(q.arrival < r.arrival and r.admitted < q.finished for q in served for r in served)
    summary = serving.latency_summary(served)
    assert summary["n"] == len(reqs) and summary["p99_ms"] >= summary["p50_ms"] > 0


def _oracle_key(sc):
    """What the oracle gives a request: status, value-volume digest, goal and
    plan (the same key as _key)."""
    import hashlib

    import oracle
    from tests.common import problem_of

    prob = problem_of(sc)
    B = oracle.render(prob, sc.image, *sc.vehicle)
    V = oracle.init(prob, B, sc.start)
    oracle.cycles(prob, B, V, sc.n_cycles)
    digest = hashlib.sha1(V.tobytes()).hexdigest()
    try:
        best, score = oracle.goal_search(prob, B, V, sc.goal, sc.goal_radius, sc.w_xy, sc.w_t)
        steps = oracle.backtrack(prob, B, V, sc.start, best)
    except oracle.OracleError as e:
        return (e.rc, digest, None, None)
    value = int(V[best[2], best[1], best[0]])
    return (0, digest, (best, value, score), [(s.maneuver, s.steps, s.frm, s.to, s.cost) for s in steps])


def test_served_results_match_oracle():
    """Small and large requests (a 512-side request among them) admitted
    under a budget that makes requests wait, by both admission paths, with
    ticks small enough that plans are picked in turn (shortest remaining
    work first) and share launches at different points of their schedules:
    every served result equals the oracle's."""
    import os

    import oracle

    oracle.set_threads(min(16, os.cpu_count() or 1))
    rng = np.random.default_rng(78)
    reqs = [scenes.random_instance(rng, sides=(64, 128), thetas=(64, 128), n_range=(2, 5), name="s%02d" % k)
            for k in range(6)]
    reqs.insert(1, scenes.random_instance(rng, sides=(512,), thetas=(128,), n_range=(3, 3), name="L512"))
    reqs.insert(4, scenes.random_instance(rng, sides=(256,), thetas=(256,), n_range=(3, 3), name="L256"))
    arrivals = [0.0] * len(reqs)  # all at once: the budget below admits the 512-side plan and one more at most
    budget = serving.footprint_bytes(reqs[1]) + min(serving.footprint_bytes(sc) for sc in reqs)
    srv = serving.Server(budget, max_live=8, digests=True, fill_poses=1 << 22, tick_poses=1 << 21)
    served = srv.run(reqs, arrivals)
    srv.close()
    assert srv.admission_waits > 0 and srv.ticks > len(reqs)
    # both admission paths ran: by the scheduling thread while no sweeps were
    # queued (the first requests), by the admission thread behind running sweeps
    assert 0 < srv.admitted_inline < len(reqs)
    for sc, r in zip(reqs, served):
        print("request %s %dx%dx%d N=%d: oracle" % (sc.name, sc.nx, sc.nx, sc.nt, sc.n_cycles), flush=True)
        assert _key(r) == _oracle_key(sc), sc.name
