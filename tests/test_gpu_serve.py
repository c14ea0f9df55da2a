"""Serving: requests that arrive while others run are admitted into the
running batch as memory frees up; each result equals the same request run
alone, bit for bit."""

import numpy as np
import pytest

import oracle
from paper_1606_07801_amd import flb, serve
from tests.gpu_common import RTOL, report, scaled_error

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
    # the served results of the requests at mean density >= 5 against the
    # oracle's FP64 run of the same request from the same initial state
    checked = 0
    for r in S.finished:
        if r.rho < 5.0:
            continue
        lat = oracle.make_lattice(r.d)
        w32 = flb.constants(r.d)[0].astype(np.float32)
        f0 = np.broadcast_to((w32 * np.float32(r.rho)).reshape((-1,) + (1,) * r.d),
                             (lat.Q,) + tuple(reversed(r.dims))).astype(np.float64)
        fo = oracle.run(f0, oracle.Params(d=r.d, omega_j=r.omega, seed=r.seed), r.steps)
        err = scaled_error(r.result["state"], fo, r.rho, lat.w)
        assert report(f"served request {r.id} D{r.d} {r.dims} {r.steps} steps", err) <= RTOL[4]
        checked += 1
    assert checked >= 4


def test_oversized_request_rejected():
    r = serve.Request(0, 0.0, 2, (512, 512), 10, 1.0, 5.0, 1)
    S = serve.Server(budget_bytes=1 << 20)
    S.run([r])
    assert S.rejected == [r] and r.error
    S.close()
