"""Host logic of the continuous-batching server, with a stand-in batch (no
GPU): HBM-budget admission in arrival order, rejection of requests larger
than the budget, tick sizes bounded by the smallest remaining step count,
retirement releasing memory, and the latency summary."""

import pytest

from paper_1606_07801_amd import serve


class FakeBatch:
    def __init__(self, **kw):
        self.members, self.steps = [], []

    def admit(self, lat):
        self.members.append(lat)

    def retire(self, lat):
        self.members.remove(lat)

    def step(self, n):
        self.steps.append((n, len(self.members)))

    def sync(self):
        pass

    def close(self):
        pass


@pytest.fixture
def fake(monkeypatch):
    started, finished = [], []

    def start(torch, req, device):
        req.lat = object()
        started.append(req.id)

    def finish(req):
        finished.append(req.id)
        req.result = {"id": req.id}
        req.lat = None

    monkeypatch.setattr(serve.flb, "Batch", FakeBatch)
    monkeypatch.setattr(serve, "start_request", start)
    monkeypatch.setattr(serve, "finish_request", finish)
    monkeypatch.setattr(serve, "request_bytes", lambda req: req.sites * 100)
    return started, finished


def _req(i, sites, steps):
    return serve.Request(i, 0.0, 1, (sites,), steps, 1.0, 10.0, i)


def test_admission_by_budget_and_order(fake):
    started, finished = fake
    S = serve.Server(budget_bytes=100 * 250, tick_steps=64, device="cpu")
    reqs = [_req(0, 100, 100), _req(1, 100, 30), _req(2, 100, 50), _req(3, 300, 10)]
    for r in reqs:
        S.submit(r)
    assert [r.id for r in S.rejected] == [3]          # 300 sites need more than the budget
    S.tick(0.0)
    assert started == [0, 1]                           # request 2 does not fit yet
    assert S.batch.steps[-1] == (30, 2)                # bounded by the smallest remaining count
    assert 1 in finished and S.used == 100 * 100       # request 1 retired, memory released
    S.tick(1.0)
    assert started == [0, 1, 2]
    while S.active or S.queue:
        S.tick(2.0)
    assert sorted(finished) == [0, 1, 2]
    assert S.used == 0
    assert S.site_updates == 100 * 100 + 100 * 30 + 100 * 50


def test_zero_step_request_retires_at_admission(fake):
    started, finished = fake
    S = serve.Server(budget_bytes=10 ** 6, device="cpu")
    S.submit(_req(0, 10, 0))
    S.tick(0.0)
    assert finished == [0] and not S.active and S.ticks == 0


def test_summary_percentiles(fake):
    S = serve.Server(budget_bytes=10 ** 9, device="cpu")
    for i in range(10):
        r = _req(i, 10, 5)
        r.arrival, r.done = 0.0, float(i + 1)
        S.finished.append(r)
    S.site_updates = 5 * 10 ** 8
    out = serve.summary(S, 10.0)
    assert out["requests"] == 10 and out["p50_latency_s"] == pytest.approx(5.5)
    assert out["p99_latency_s"] == pytest.approx(9.91, abs=1e-4) and out["mlups"] == pytest.approx(50.0)
