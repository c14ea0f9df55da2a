"""Pins of the oracle's lattices with spatially varying temperature or rates
(Sec. IV, non-homogeneous systems, and the averaged diffusion equation
eq. DiffAve).

f_i = w_i(theta(x)) rho(x) with theta(x) rho(x) constant is a fixed point of
the step for any rates: the collision leaves an equilibrium unchanged, and
every moving population arriving at x carries theta/2 times theta rho of its
origin, the same constant.  So the stationary state has theta rho uniform
(two temperatures: the paper's <rho_1 theta_1> = <rho_2 theta_2>) and, for
equal theta and different rates, a uniform density (the Ito-Stratonovich
case)."""

import numpy as np
import pytest

import oracle


def _halves(shape):
    region = np.zeros(shape[::-1], dtype=np.uint8)
    region[..., shape[0] // 2:] = 1
    return region


def test_single_region_equals_uniform_step():
    gen = np.random.default_rng(2)
    f = gen.poisson(3.0, size=(5, 6, 9)).astype(np.float64)
    p = oracle.Params(d=2, omega_j=1.3, seed=4)
    a = oracle.run(f, p, 7)
    b = oracle.run_regions(f, [p], np.zeros((6, 9), dtype=np.uint8), 7)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("omega", [1.0, 0.7, 1.3])
def test_two_temperatures_stationary_theta_rho(omega):
    L = 40
    p1 = oracle.Params(d=1, theta=1 / 3, omega_j=omega, noise="off")
    p2 = oracle.Params(d=1, theta=1 / 6, omega_j=omega, noise="off")
    lat = oracle.make_lattice(1)
    f = lat.w[:, None] * np.full(L, 10.0)[None, :]
    region = _halves((L,))
    f = oracle.run_regions(f, [p1, p2], region, 16000)
    rho = f.sum(axis=0)
    theta = np.where(region == 0, 1 / 3, 1 / 6)
    u = theta * rho
    assert np.abs(u / u.mean() - 1).max() < 1e-9
    assert abs(rho.sum() - 10.0 * L) < 1e-9
    assert abs(rho[region == 1].mean() / rho[region == 0].mean() - 2.0) < 1e-9


@pytest.mark.parametrize("d,shape", [(1, (30,)), (2, (16, 6))])
def test_two_rates_stationary_uniform_density(d, shape):
    # D = (1/omega - 1/2) theta: 1/30 and 1/3 at theta = 1/3
    p1 = oracle.Params(d=d, omega_j=1 / 0.6, noise="off")
    p2 = oracle.Params(d=d, omega_j=1 / 1.5, noise="off")
    lat = oracle.make_lattice(d)
    x = np.arange(shape[0])
    rho0 = 10.0 + 3.0 * np.cos(2 * np.pi * x / shape[0])
    rho0 = np.broadcast_to(rho0, shape[::-1])
    f = lat.w.reshape((-1,) + (1,) * d) * rho0[None]
    f = oracle.run_regions(f, [p1, p2], _halves(shape), 8000)
    rho = f.sum(axis=0)
    assert np.abs(rho / 10.0 - 1).max() < 1e-8


def test_regions_conserve_mass_with_noise():
    gen = np.random.default_rng(3)
    f = gen.poisson(8.0, size=(5, 7, 11)).astype(np.float64)
    plist = [oracle.Params(d=2, theta=th, omega_j=om, seed=9) for th, om in ((1 / 3, 1.0), (0.2, 1.7), (0.25, 0.6))]
    region = gen.integers(0, 3, size=(7, 11)).astype(np.uint8)
    g = oracle.run_regions(f, plist, region, 20)
    assert abs(g.sum() - f.sum()) < 1e-9 * f.sum()
