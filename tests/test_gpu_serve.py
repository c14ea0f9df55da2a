"""Serving: requests that arrive while others run are admitted into the
running batch as memory frees up; each result equals the same request run
alone, bit for bit."""

import numpy as np
import pytest

from paper_1606_07801_amd import flb, serve

pytestmark = pytest.mark.gpu


def _requests():
    gen = np.random.default_rng(3)
    specs = [(1, (64,)), (1, (3000,)), (1, (50000,)), (2, (200, 150)), (2, (64, 64)), (3, (30, 20, 10)),
             (2, (513, 31)), (1, (777,)), (3, (16, 16, 16)), (2, (128, 128))]
    out = []
    for i, (d, dims) in enumerate(specs):
        out.append(serve.Request(i, arrival=0.004 * i, d=d, dims=dims, steps=int(gen.integers(5, 120)),
                                 omega=float(gen.uniform(0.5, 1.9)), rho=float(gen.uniform(0.1, 50)),
                                 seed=1000 + i, precision=4, keep_state=True))
    return out


def test_served_results_equal_alone():
    import torch
    reqs = _requests()
    # budget for about three requests at a time: forces queueing and refills
    budget = 3 * max(serve.request_bytes(r) for r in reqs)
    S = serve.Server(budget_bytes=budget, tick_steps=16, chunk=8)
    S.run(reqs)
    assert len(S.finished) == len(reqs) and not S.rejected
    assert S.used == 0
    for r in S.finished:
        assert r.result["steps"] == r.steps
        alone = flb.Lattice(r.d, r.dims, precision=4, omega=r.omega, seed=r.seed)
        alone.set_populations(serve.initial_state(torch, r, S.device))
        alone.step(r.steps)
        ref = alone.get_populations()
        alone.close()
        assert np.array_equal(r.result["state"], ref), r.id
        assert r.done >= r.arrival
    s = serve.summary(S, 1.0)
    assert s["requests"] == len(reqs)
    S.close()


def test_oversized_request_rejected():
    r = serve.Request(0, 0.0, 2, (512, 512), 10, 1.0, 5.0, 1)
    S = serve.Server(budget_bytes=1 << 20)
    S.run([r])
    assert S.rejected == [r] and r.error
    S.close()
