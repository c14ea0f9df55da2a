"""Two D2Q5 steps per pass (kernel "two"): the state is bit-identical to
single steps of the flat kernel on ragged and degenerate boxes, across the
2^32 wrap of the noise counter's step word and with every sampling kind
interleaved (a pair is fused only when nothing is sampled between its
steps); one case against the oracle."""

import numpy as np
import pytest

import oracle
from tests.gpu_common import RTOL, gpu_lattice, poisson_state, report, scaled_error

pytestmark = pytest.mark.gpu

DIMS = [(300, 70), (256, 8), (513, 33), (5, 3), (1, 7), (1000, 1), (64, 64)]


def _run(dims, precision, kernel, steps, t0, ty=0, nt=0, sample=False, noise="local", law="gauss"):
    dt = np.float32 if precision == 4 else np.float64
    f0 = poisson_state(2, dims, 10.0, seed=4).astype(dt)
    L = gpu_lattice(2, dims, precision, omega=1.3, omega_n=0.8, seed=99, kernel=kernel, tile_rows=ty,
                    nt_store=nt, noise=noise, law=law)
    L.set_populations(f0, step=t0)
    out = {}
    if sample:
        L.set_moment_sampling(5)
        L.set_sampling(3, [[1, 0], [0, 1], [1, 1]])
        L.set_correlation(7, [[1, 0], [2, 1]], 2)
    L.step(steps)
    out["f"] = L.get_populations()
    out["t"] = L.t
    if sample:
        out["mom"] = L.sampled_moments()
        out["sk"] = L.structure_factor(mode="read")[:3]
        out["corr"] = L.correlation()
    L.close()
    return out


@pytest.mark.parametrize("precision", [4, 8])
@pytest.mark.parametrize("dims", DIMS)
def test_two_step_bit_identical(dims, precision):
    t0 = (1 << 32) - 3                    # a pair straddles the wrap of the step word
    ref = _run(dims, precision, "flat", 13, t0, ty=2, nt=1)
    for ty, nt in ((8, 1), (2, 0), (4, 1), (16, 0)):
        got = _run(dims, precision, "two", 13, t0, ty=ty, nt=nt)
        assert got["t"] == ref["t"] == t0 + 13
        assert np.array_equal(got["f"].view(np.uint8), ref["f"].view(np.uint8)), (ty, nt)


@pytest.mark.parametrize("precision", [4, 8])
@pytest.mark.parametrize("noise,law", [("global", "gauss"), ("local", "uniform"), ("off", "gauss"),
                                       ("global", "uniform")])
def test_two_step_other_noise_plans(noise, law, precision):
    # local Gaussian noise runs instances with the noise plan fixed at compile
    # time; every other combination reads it from the parameters
    dims = (300, 70)
    ref = _run(dims, precision, "flat", 9, 5, ty=2, nt=1, noise=noise, law=law)
    for ty, nt in ((8, 1), (4, 0)):
        got = _run(dims, precision, "two", 9, 5, ty=ty, nt=nt, noise=noise, law=law)
        assert np.array_equal(got["f"].view(np.uint8), ref["f"].view(np.uint8)), (ty, nt)
    for ty in (8, 16):  # and against the fixed plan's instances: the noise changes the state
        if noise != "local" or law != "gauss":
            loc = _run(dims, precision, "two", 9, 5, ty=ty, nt=1)
            assert not np.array_equal(loc["f"], ref["f"])


def test_two_step_with_sampling():
    ref = _run((300, 70), 8, "flat", 40, 1, ty=2, sample=True)
    got = _run((300, 70), 8, "two", 40, 1, ty=8, sample=True)
    assert np.array_equal(got["f"], ref["f"])
    assert got["mom"][1] == ref["mom"][1] and np.array_equal(got["mom"][0]["sum_ff"], ref["mom"][0]["sum_ff"])
    assert np.array_equal(got["sk"], ref["sk"])
    assert got["corr"][2] == ref["corr"][2] and np.array_equal(got["corr"][0], ref["corr"][0])


def test_two_step_matches_oracle():
    dims = (300, 70)
    f0 = poisson_state(2, dims, 10.0, seed=4)
    L = gpu_lattice(2, dims, 8, omega=1.3, omega_n=0.8, seed=99, kernel="two", tile_rows=8)
    L.set_populations(f0)
    L.step(10)
    g = L.get_populations()
    L.close()
    fo = oracle.run(f0, oracle.Params(d=2, omega_j=1.3, omega_n=0.8, seed=99), 10)
    w = oracle.make_lattice(2).w
    assert report("two-step D2 (300, 70) fp64", scaled_error(g, fo, 10.0, w)) <= RTOL[8]


@pytest.mark.parametrize("precision", [4, 8])
def test_sampled_pairs_equal_single_steps(precision):
    # axis-only k-list: the sampled step is fused into a pair whose pass also
    # writes the density partials; state and S(k) sums equal the one-step path
    dims = (300, 70)
    ks = [[1, 0], [0, 1], [5, 0], [0, 7], [0, 0]]
    out = []
    for kern, ty in (("flat", 2), ("two", 8)):
        dt = np.float32 if precision == 4 else np.float64
        f0 = poisson_state(2, dims, 10.0, seed=4).astype(dt)
        L = gpu_lattice(2, dims, precision, seed=3, kernel=kern, tile_rows=ty, nt_store=1)
        L.set_populations(f0)
        L.set_sampling(4, ks)
        L.step(23)
        out.append((L.get_populations(), L.structure_factor(mode="read")[:len(ks)]))
        L.close()
    assert np.array_equal(out[0][0].view(np.uint8), out[1][0].view(np.uint8))
    assert np.array_equal(out[0][1], out[1][1])
