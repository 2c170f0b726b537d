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
