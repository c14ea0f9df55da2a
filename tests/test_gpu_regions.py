"""Lattices whose temperature or rates vary by region (Sec. IV,
non-homogeneous systems): parity with the oracle on the same seeded inputs,
bit identity with the uniform kernels for a single region, and the paper's
two measurements (Fig. 6) with noise: two temperatures give theta rho equal
in both domains, two diffusion constants leave the density uniform."""

import numpy as np
import pytest

import oracle
from paper_1606_07801_amd import flb
from tests.gpu_common import RTOL, gpu_lattice, poisson_state, report, scaled_error

pytestmark = pytest.mark.gpu



def _setup(d):
    th = {1: (1 / 3, 0.2, 0.45), 2: (1 / 3, 0.2, 0.25), 3: (0.25, 0.15, 0.3)}[d]
    om = ((1.0, 0.0, 0.0), (1.7, 0.9, 1.3), (0.6, 0.0, 0.0))
    return th, om


@pytest.mark.parametrize("noise,law", [("local", "gauss"), ("global", "uniform")])
@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("d,dims", [(1, (1000,)), (2, (300, 70)), (3, (40, 33, 17))])
def test_regions_match_oracle(d, dims, precision, noise, law):
    # FP32 at a mean density where no site comes near rho = 0 within the run
    # (there the amplitude sqrt(max(rho, 0)) magnifies FP32 rounding)
    dt = np.float32 if precision == 4 else np.float64
    rho = 40.0 if precision == 4 else 10.0
    f0 = poisson_state(d, dims, rho, seed=6).astype(dt)
    region = np.random.default_rng(8).integers(0, 3, size=dims[::-1]).astype(np.uint8)
    th, om = _setup(d)
    L = gpu_lattice(d, dims, precision, seed=12, noise=noise, law=law)
    L.set_populations(f0)
    L.set_regions(region, th, om)
    L.step(25)
    g = L.get_populations()
    L.close()
    plist = [oracle.Params(d=d, theta=th[r], omega_j=om[r][0], omega_n=om[r][1], omega_s=om[r][2], seed=12,
                           noise=noise, law=law) for r in range(3)]
    fo = oracle.run_regions(f0.astype(np.float64), plist, region, 25)
    w = np.full(2 * d + 1, 0.5 * max(th))
    err = report(f"regions D{d} {dims} fp{8 * precision} {noise}/{law}", scaled_error(g, fo, rho, w))
    assert err <= RTOL[precision]


@pytest.mark.parametrize("d,dims", [(1, (1000,)), (2, (300, 70))])
def test_single_region_bit_identical_to_uniform(d, dims):
    f0 = poisson_state(d, dims, 10.0, seed=2)
    outs = []
    for use_regions in (False, True):
        L = gpu_lattice(d, dims, 8, omega=1.3, omega_n=0.8, seed=5, kernel="plain")
        L.set_populations(f0)
        if use_regions:
            L.set_regions(np.zeros(dims[::-1], dtype=np.uint8), [1 / 3], [(1.3, 0.8, 0.0)])
        L.step(11)
        outs.append(L.get_populations())
        L.close()
    assert np.array_equal(outs[0].view(np.uint8), outs[1].view(np.uint8))


def test_regions_errors():
    L = gpu_lattice(2, (8, 4), 8)
    reg = np.zeros((4, 8), dtype=np.uint8)
    reg[0, 0] = 2
    with pytest.raises(flb.FlbError) as e:
        L.set_regions(reg, [1 / 3, 0.2], [1.0, 1.0])           # index beyond nregions
    assert e.value.code == flb.FLB_EINVAL
    with pytest.raises(flb.FlbError):
        L.set_regions(np.zeros((4, 8)), [0.6], [1.0])         # theta >= 1/d
    with pytest.raises(flb.FlbError):
        L.set_regions(np.zeros((4, 8)), [0.3], [2.0])         # omega outside (0, 2)
    L.set_regions(np.zeros((4, 8)), [0.3], [1.0])
    B = flb.Batch()
    with pytest.raises(flb.FlbError) as e:
        B.admit(L)
    assert e.value.code == flb.FLB_EINVAL
    L.set_regions(None)
    B.admit(L)
    B.retire(L)
    B.close()
    L.close()


def _two_domain_profile(theta, omega, steps=20_000, every=50, nsamp=200, side=64, rho=100.0):
    d = 2
    lat = oracle.make_lattice(d)
    f0 = poisson_state(d, (side, side), rho, seed=3)
    region = np.zeros((side, side), dtype=np.uint8)
    region[:, side // 2:] = 1
    L = gpu_lattice(d, (side, side), 8, seed=31)
    L.set_populations(f0)
    L.set_regions(region, theta, omega)
    L.step(steps)
    acc = np.zeros(side)
    for _ in range(nsamp):
        L.step(every)
        acc += L.profile(0)[0] / side
    L.close()
    del lat
    return acc / nsamp


def test_two_temperatures_fig6a():
    # theta = 1/3 | 1/6, unit rates: <rho_1 theta_1> = <rho_2 theta_2>
    m = _two_domain_profile((1 / 3, 1 / 6), (1.0, 1.0))
    a, b = m[4:28].mean(), m[36:60].mean()
    print(f"[fig6a] rho(theta=1/3) {a:.3f}  rho(theta=1/6) {b:.3f}  ratio {b / a:.4f}", flush=True)
    assert abs(b / a - 2.0) < 0.01
    # flat inside each domain, also next to the interfaces
    assert np.abs(m[:32] / a - 1).max() < 0.02 and np.abs(m[32:] / b - 1).max() < 0.02


def test_two_diffusion_constants_fig6b():
    # D = 1/30 | 1/3 (omega_j = 1/0.6 | 1/1.5 at theta = 1/3): uniform density
    m = _two_domain_profile((1 / 3, 1 / 3), (1 / 0.6, 1 / 1.5))
    print(f"[fig6b] rho left {m[:32].mean():.3f} right {m[32:].mean():.3f}  max dev {np.abs(m / 100 - 1).max():.4f}",
          flush=True)
    assert abs(m[:32].mean() / m[32:].mean() - 1) < 0.01
    assert np.abs(m / 100.0 - 1).max() < 0.02
