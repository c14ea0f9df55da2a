"""The density profile on the GPU path and the paper's non-equilibrium test
(Sec. IV, non-equilibrium dynamics: a block of low density in a periodic
strip, averaged over y; Figs. 8 and 9, eq. rhoth).

At unit rates the collision maps every population to w_i rho, and with
local noise of variance rho (w_i delta_ij - w_i w_j) a Poisson covariance
stays Poisson (diagonal, equal to the means) for any mean, in or out of
equilibrium.  So with Poisson initial counts the density variance equals
the mean density at every x and t, which is eq. (rhoth); and because the
noise has zero mean and the update is linear, the mean profile is exactly
the noise-off evolution of the initial state (here taken from the oracle on
a one-row lattice, y-averaged populations).  Global noise breaks the first
identity: its amplitude follows the mean density of the whole lattice."""

import numpy as np
import pytest

import oracle
from paper_1606_07801_amd import experiments, inputs
from tests import closed_forms as cf
from tests.gpu_common import gpu_lattice, poisson_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("d,dims", [(1, (1000,)), (2, (300, 70)), (3, (40, 33, 17))])
def test_profile_matches_oracle(d, dims, precision):
    dt = np.float32 if precision == 4 else np.float64
    f0 = poisson_state(d, dims, 7.0, seed=9).astype(dt)
    L = gpu_lattice(d, dims, precision, seed=1)
    L.set_populations(f0)
    for axis in range(d):
        s, s2 = L.profile(axis)
        r, r2 = oracle.profile(f0.astype(np.float64), axis)
        assert np.abs(s - r).max() <= 1e-13 * np.abs(r).max()
        assert np.abs(s2 - r2).max() <= 1e-13 * np.abs(r2).max()
    L.close()


NX, NY, RHO_IN, RHO_OUT, TIMES = 100, 10_000, 20.0, 120.0, (100, 400, 1600)


def _front(noise):
    lat = oracle.make_lattice(2)
    rho0 = inputs.block_profile(NX, RHO_IN, RHO_OUT)
    lam = lat.w[:, None, None] * np.broadcast_to(rho0[None, :], (NY, NX))[None]
    f0 = inputs.poisson_sites(lam, seed=17)
    return f0, experiments.diffusion_front(NX, NY, RHO_IN, RHO_OUT, TIMES, omega=1.0, noise=noise, seed=17,
                                           precision=8, f0=f0)


def test_front_mean_and_variance_local_noise():
    f0, out = _front("local")
    # expected mean: the noise-off oracle on the y-averaged populations (one row)
    fbar = f0.mean(axis=1, keepdims=True)
    p = oracle.Params(d=2, omega_j=1.0, seed=0, noise="off")
    prev = 0
    for t, m, v in zip(out["times"], out["mean"], out["var"]):
        fbar = oracle.run(fbar, p, t - prev, t0=prev)
        prev = t
        expect = fbar.sum(axis=0)[0]
        sig = np.sqrt(v / NY)
        z = (m - expect) / sig
        # eq. (rhoth): variance over y = mean; relative sd of a variance
        # estimate from NY Gaussian-like samples is sqrt(2 / NY)
        r = v / m
        zr = (r - 1) / np.sqrt(2.0 / NY)
        theory = cf.front_profile(NX, t, 1.0 / 6.0, RHO_IN, RHO_OUT)
        print(f"[front] t={t}: mean max |z| {np.abs(z).max():.2f}; var/mean {r.mean():.4f} "
              f"(min {r.min():.3f} max {r.max():.3f}, max |z| {np.abs(zr).max():.2f}); "
              f"|mean - erf| max {np.abs(m - theory).max():.3f}", flush=True)
        assert np.abs(z).max() < 5.0
        assert abs(r.mean() - 1) < 0.005
        assert np.abs(zr).max() < 5.0
        # the continuum erf series of the paper, with the lattice D = theta/2
        assert np.abs(m - theory).max() < 0.005 * (RHO_OUT - RHO_IN)


def test_front_variance_global_noise():
    # the amplitude follows the lattice-wide mean density (70), so the
    # variance no longer tracks the local mean: above it in the low-density
    # block, below it outside
    _, out = _front("global")
    m, v = out["mean"][-1], out["var"][-1]
    inner = slice(NX // 4 + 10, 3 * NX // 4 - 10)
    outer = np.r_[0:NX // 4 - 10, 3 * NX // 4 + 10:NX]
    ri, ro = (v / m)[inner].mean(), (v / m)[outer].mean()
    print(f"[front] global noise t={out['times'][-1]}: var/mean inside {ri:.3f}, outside {ro:.3f}", flush=True)
    assert ri > 1.1 and ro < 0.95
