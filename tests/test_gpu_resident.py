"""The resident kernel (a whole small lattice in one workgroup's LDS, many
steps per launch): its state is bit-identical to the HBM kernels', its
sampled statistics equal the HBM path's to rounding, the step counter and
the sample counts carry across launches, and it refuses lattices that do
not fit."""

import numpy as np
import pytest

from paper_1606_07801_amd import flb
from tests.gpu_common import gpu_lattice, poisson_state

pytestmark = pytest.mark.gpu

# (d, dims): 1, 2 and 4 sites per thread; ragged widths
CASES = [(1, (256,)), (1, (1000,)), (1, (2500,)), (2, (10, 10)), (2, (37, 23)), (2, (45, 40)),
         (3, (5, 4, 3)), (3, (12, 10, 9))]


def _run(d, dims, precision, kernel, steps, t0=0, sample=False, noise="local", law="gauss", seed=7):
    dt = np.float32 if precision == 4 else np.float64
    f0 = poisson_state(d, dims, 10.0, seed=5).astype(dt)
    L = gpu_lattice(d, dims, precision, omega=1.3, omega_n=0.7, seed=seed, noise=noise, law=law, kernel=kernel)
    L.set_populations(f0, step=t0)
    out = {}
    if sample:
        ks = [[0] * d, [1] + [0] * (d - 1), [2] * d, [-1] + [3] * (d - 1), [dims[0] - 1] + [0] * (d - 1)]
        L.set_moment_sampling(3)
        L.set_sampling(2, ks)
        L.set_correlation(2, ks, 5)
    L.step(steps)
    out["f"] = L.get_populations()
    out["t"] = L.t
    if sample:
        out["mom"], out["nmom"] = L.sampled_moments()
        out["sk"] = L.structure_factor(mode="read")[:5]
        out["sij"], out["ct"], out["ncorr"] = L.correlation()
    L.close()
    return out


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("d,dims", CASES)
def test_resident_state_bit_identical(d, dims, precision):
    # starts 5 steps below 2^32: the noise counter's step word wraps inside
    a = _run(d, dims, precision, "resident", 37, t0=(1 << 32) - 5)
    b = _run(d, dims, precision, "flat", 37, t0=(1 << 32) - 5)
    assert a["t"] == b["t"] == (1 << 32) + 32
    assert np.array_equal(a["f"].view(np.uint8), b["f"].view(np.uint8))


@pytest.mark.parametrize("noise,law", [("global", "uniform"), ("off", "gauss")])
def test_resident_noise_modes(noise, law):
    a = _run(2, (37, 23), 8, "resident", 20, noise=noise, law=law)
    b = _run(2, (37, 23), 8, "plain", 20, noise=noise, law=law)
    assert np.array_equal(a["f"], b["f"])


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("d,dims", [(1, (256,)), (1, (1000,)), (2, (37, 23)), (2, (32, 16)), (3, (12, 10, 9)),
                                    (3, (8, 4, 16))])
def test_resident_sampling_equals_hbm_path(d, dims, precision):
    # power-of-two axes take the FFT of the marginal, the others a DFT
    a = _run(d, dims, precision, "resident", 23, t0=1, sample=True)
    b = _run(d, dims, precision, "flat", 23, t0=1, sample=True)
    assert np.array_equal(a["f"], b["f"])
    assert a["nmom"] == b["nmom"] == 7 and a["ncorr"] == b["ncorr"] == 11
    for key in ("mass", "sum_rho2", "sum_rho_pos"):
        assert abs(a["mom"][key] - b["mom"][key]) <= 1e-13 * abs(b["mom"][key])
    assert a["mom"]["n_negative"] == b["mom"]["n_negative"] and a["mom"]["nonfinite"] == 0
    assert np.abs(a["mom"]["sum_ff"] - b["mom"]["sum_ff"]).max() <= 1e-13 * np.abs(b["mom"]["sum_ff"]).max()
    assert np.abs(a["sk"] - b["sk"]).max() <= 1e-11 * np.abs(b["sk"]).max()
    sc = np.abs(b["sij"]).max()
    assert np.abs(a["sij"] - b["sij"]).max() <= 1e-13 * sc
    assert np.abs(a["ct"] - b["ct"]).max() <= 1e-13 * np.abs(b["ct"]).max()
    print(f"[resident] D{d} {dims} fp{8 * precision}: S(k) rel {np.abs(a['sk'] - b['sk']).max() / np.abs(b['sk']).max():.1e}",
          flush=True)


def test_resident_many_launches():
    # more steps than one launch takes: state, step and sample counts carry over
    a = _run(3, (5, 4, 3), 8, "resident", 70001, sample=False)
    b = _run(3, (5, 4, 3), 8, "plain", 70001, sample=False)
    assert a["t"] == b["t"] == 70001
    assert np.array_equal(a["f"], b["f"])
    L = gpu_lattice(1, (64,), 8, kernel="resident")
    L.set_populations(poisson_state(1, (64,), 5.0, seed=1))
    L.set_moment_sampling(7)
    L.step(70000)
    assert L.sampled_moments()[1] == len(range(0, 70000, 7))
    L.close()


def test_resident_refuses_what_does_not_fit():
    with pytest.raises(flb.FlbError) as e:
        gpu_lattice(2, (100, 100), 8, kernel="resident")
    assert e.value.code == flb.FLB_EINVAL
