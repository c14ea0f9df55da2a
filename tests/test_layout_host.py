"""The single-buffer AA layout on the host: it needs half the population
memory of two buffers, the same workspace, and is refused with the kernels
that need a second buffer; the server's layout policy."""

import pytest

from paper_1606_07801_amd import flb, serve


@pytest.mark.parametrize("d,dims", [(1, (1000,)), (2, (300, 70)), (3, (40, 33, 17))])
@pytest.mark.parametrize("precision", [4, 8])
def test_aa_needs_half_the_population_memory(d, dims, precision):
    two = flb.required_bytes(flb.make_params(d, dims, precision))
    aa = flb.required_bytes(flb.make_params(d, dims, precision, layout="aa"))
    n = 1
    for x in dims:
        n *= x
    assert two[0] == 2 * (2 * d + 1) * n * precision
    assert aa[0] * 2 == two[0] and aa[1] == two[1]


@pytest.mark.parametrize("kernel", ["two", "rows", "plain"])
def test_aa_refuses_kernels_that_need_two_buffers(kernel):
    with pytest.raises(flb.FlbError) as e:
        flb.required_bytes(flb.make_params(2, (64, 64), 4, kernel=kernel, layout="aa"))
    assert e.value.code == flb.FLB_EINVAL


def test_aa_refuses_planes_beyond_32_bit_offsets():
    # Q N precision >= 2^32: the flat kernel's 32-bit offsets do not reach
    with pytest.raises(flb.FlbError):
        flb.required_bytes(flb.make_params(2, (16384, 16384), 4, layout="aa"))
    flb.required_bytes(flb.make_params(2, (16384, 13107), 4, layout="aa"))


def test_unknown_layout_refused():
    p = flb.make_params(2, (8, 8), 4)
    p.layout = 2
    with pytest.raises(flb.FlbError):
        flb.required_bytes(p)


def test_server_layout_policy():
    def req(d, side):
        return serve.Request(0, 0.0, d, (side,) * d, 10, 1.0, 5.0, 1)
    # auto: the faster layout per model (one buffer for D1Q3, two for D2Q5
    # and D3Q7), "aa": one buffer for every request that can take it
    assert serve.pick_layout(req(2, 500), "auto") == "two"
    assert serve.pick_layout(req(1, 5000), "auto") == "aa"
    assert serve.pick_layout(req(3, 100), "auto") == "two"
    assert serve.pick_layout(req(2, 500), "aa") == "aa"
    assert serve.pick_layout(req(3, 100), "two") == "two"
    # beyond the flat kernel's 32-bit plane offsets: two buffers whatever the policy
    assert serve.pick_layout(req(3, 800), "aa") == "two"
    r = req(3, 100)
    r.layout = "aa"
    a = serve.request_bytes(r)
    r.layout = "two"
    assert serve.request_bytes(r) - a == 7 * 100 ** 3 * 4
    assert serve.fallback_bytes(r, "auto") == a and serve.fallback_bytes(r, "two") is None
    big = req(3, 800)
    assert serve.fallback_bytes(big, "auto") is None


class _Batch:
    def __init__(self, **kw):
        self.members = []

    def admit(self, lat):
        self.members.append(lat)

    def retire(self, lat):
        self.members.remove(lat)

    def step(self, n):
        pass

    def sync(self):
        pass

    def close(self):
        pass


def test_auto_policy_falls_back_to_one_buffer_under_pressure(monkeypatch):
    # two D3Q7 requests whose two-buffer footprints do not fit together: the
    # second is admitted at once in the AA layout instead of waiting
    monkeypatch.setattr(serve.flb, "Batch", _Batch)
    monkeypatch.setattr(serve, "start_request", lambda torch, req, dev: setattr(req, "lat", object()))
    monkeypatch.setattr(serve, "finish_request", lambda req: setattr(req, "result", {}))
    sizes = {"two": 1000, "aa": 600}
    monkeypatch.setattr(serve, "request_bytes", lambda req: sizes[req.layout])
    for policy, layouts in (("auto", ["two", "aa"]), ("two", ["two"])):
        S = serve.Server(budget_bytes=1700, tick_steps=8, device="cpu", layout=policy)
        reqs = [serve.Request(i, 0.0, 3, (40, 40, 40), 100, 1.0, 5.0, i) for i in range(2)]
        for r in reqs:
            S.submit(r)
        S.tick(0.0)
        assert [r.layout for r in S.active] == layouts
        assert S.used == sum(sizes[lay] for lay in layouts)
        assert S.fallbacks == (1 if policy == "auto" else 0)
