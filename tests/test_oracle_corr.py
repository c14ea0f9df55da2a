"""Pins of the oracle's population Fourier sums and correlators (Sec. IV:
the Fourier test, eqs. fkfk / FourierTest, and the equilibrium dynamics,
eq. TimeCorrEqn).

What fixes them independently of the oracle's own code:
* numpy's FFT (opposite kernel sign, read at -k) against the direct sum;
* the shift theorem for the paper's streaming (eq. LB) at unit rates with
  the noise off: f_i(k, t+1) = w_i exp(+2 pi i k.v_i / L) rho(k, t), and the
  explicit-scheme gain rho(k, t+1) = lambda(k) rho(k, t);
* Parseval and mass conservation;
* the stationary statistics of the linear dynamics: S_ij(k != 0) =
  N rho w_i delta_ij (eq. fkfk, no finite-size term for k != 0) and
  <rho(k, 0) rho(-k, t)> / <|rho(k)|^2> = lambda(k)^t at unit rates.
"""

import numpy as np
import pytest

import oracle
from paper_1606_07801_amd import inputs
from tests import closed_forms as cf


@pytest.mark.parametrize("dims", [(12,), (7, 5), (4, 3, 5)])
def test_amplitudes_direct_equal_fft(dims):
    d = len(dims)
    Q = 2 * d + 1
    gen = np.random.default_rng(3)
    f = gen.normal(2.0, 1.0, size=(Q,) + tuple(reversed(dims)))
    ks = gen.integers(-9, 12, size=(9, d))
    ks[0] = 0
    a = oracle.population_amplitudes(f, ks)
    b = oracle.population_amplitudes(f, ks, method="fft")
    assert np.abs(a - b).max() < 1e-11 * np.abs(f).sum()


def test_amplitude_of_one_site_has_the_paper_sign():
    # one occupied site at (x, y) = (2, 1) on a 5 x 4 box: the sum is the pure
    # phase exp(+2 pi i (2 kx / 5 + ky / 4)) -- the sign and axis order of Sec. IV
    f = np.zeros((5, 4, 5))
    f[3, 1, 2] = 2.5
    ks = np.array([[1, 0], [0, 1], [2, 3], [-1, 2]])
    a = oracle.population_amplitudes(f, ks)
    for n, (kx, ky) in enumerate(ks):
        ang = 2 * np.pi * (2 * kx / 5 + 1 * ky / 4)
        assert abs(a[n, 3] - 2.5 * (np.cos(ang) + 1j * np.sin(ang))) < 1e-14
        assert np.all(a[n, [0, 1, 2, 4]] == 0)


def test_parseval_and_mass():
    gen = np.random.default_rng(4)
    dims = (6, 4)
    f = gen.normal(1.0, 1.0, size=(5, 4, 6))
    ks = np.array([[kx, ky] for ky in range(4) for kx in range(6)])
    a = oracle.population_amplitudes(f, ks)
    lhs = np.einsum("ki,kj->ij", a, np.conj(a))
    s = oracle.lattice_sums(f)
    N = 24
    assert np.abs(lhs.imag).max() < 1e-10
    assert np.abs(lhs.real - N * s["sum_ff"]).max() < 1e-10 * N * np.abs(s["sum_ff"]).max()
    assert abs(a[0].sum() - s["mass"]) < 1e-12 * abs(s["mass"])
    del dims


@pytest.mark.parametrize("d,dims,k", [(1, (16,), (3,)), (2, (8, 6), (1, 2)), (3, (5, 4, 6), (2, 1, 1))])
def test_streaming_shift_theorem_unit_rates(d, dims, k):
    # noise off, all rates one: f*(x) = w rho(x), then f_i(x + v_i) = f*_i(x)
    lat = oracle.make_lattice(d)
    p = oracle.Params(d=d, omega_j=1.0, noise="off", seed=1)
    gen = np.random.default_rng(5)
    rho = 10 + gen.normal(0, 1, size=tuple(reversed(dims)))
    f = np.asarray(inputs.outer(lat.w, rho), dtype=np.float64)
    f1 = oracle.run(f, p, 1)
    ks = np.array([k])
    a0 = oracle.population_amplitudes(f, ks)[0]
    a1 = oracle.population_amplitudes(f1, ks)[0]
    r0 = a0.sum()
    L = np.array(dims)
    for i in range(lat.Q):
        ph = 2 * np.pi * np.sum(np.array(k) * lat.v[i] / L)
        assert abs(a1[i] - lat.w[i] * np.exp(1j * ph) * r0) < 1e-12 * np.abs(f).sum()
    lam = cf.ftcs_factor(lat.theta, k, dims)
    assert abs(a1.sum() - lam * r0) < 1e-12 * np.abs(f).sum()


def test_correlate_bookkeeping_noise_off():
    # closed forms of both sums for a single sine mode under the explicit
    # scheme: sampled every 2 steps from t0 = 3 (first sample at t = 4), 4 lags
    d, dims, k = 2, (8, 6), (1, 1)
    lat = oracle.make_lattice(d)
    p = oracle.Params(d=d, omega_j=1.0, noise="off", seed=1)
    y, x = np.meshgrid(np.arange(6), np.arange(8), indexing="ij")
    rho = 10 + 0.5 * np.cos(2 * np.pi * (x / 8 + y / 6))
    f0 = np.asarray(inputs.outer(lat.w, rho), dtype=np.float64)
    ks = np.array([k, (0, 0)])
    every, nlag, t0, nsteps = 2, 4, 3, 15
    res = oracle.correlate(f0, p, nsteps, ks, every, nlag, t0=t0)
    lam = cf.ftcs_factor(lat.theta, k, dims)
    r0 = oracle.population_amplitudes(f0, ks)[0].sum()    # rho(k, t0) = 10 * 0 + 0.5 * 48 / 2
    L = np.array(dims)
    ts = [t for t in range(t0, t0 + nsteps) if t % every == 0]
    assert res["nsamples"] == len(ts)
    sij = np.zeros((lat.Q, lat.Q), dtype=complex)
    rk = []
    for t in ts:
        r_prev = r0 * lam ** (t - t0 - 1)          # t > t0: f = w e^{i k.v} rho(t - 1)
        a = np.array([lat.w[i] * np.exp(2j * np.pi * np.sum(np.array(k) * lat.v[i] / L)) * r_prev
                      for i in range(lat.Q)])
        sij += np.outer(a, np.conj(a))
        rk.append(r0 * lam ** (t - t0))
    assert np.abs(res["sij"][0] - sij).max() < 1e-10 * abs(r0) ** 2
    for l in range(nlag):
        ct = sum(rk[s] * np.conj(rk[s + l]) for s in range(len(rk) - l))
        assert abs(res["ct"][0, l] - ct) < 1e-10 * abs(r0) ** 2
    # k = 0: every sample gives the squared mass
    M = f0.sum()
    assert abs(res["ct"][1, 0] - len(ts) * M * M) < 1e-9 * M * M
    assert abs(res["sij"][1].sum() - len(ts) * M * M) < 1e-9 * M * M


def test_stationary_population_structure_and_time_correlator():
    # eq. fkfk: S_ij(k != 0) / N = rho w_i delta_ij; eq. TimeCorrEqn at unit
    # rates: C(k, l) / C(k, 0) = lambda(k)^l (exact for the linear dynamics)
    d, dims, rho = 2, (6, 5), 40.0
    lat = oracle.make_lattice(d)
    N = 30
    p = oracle.Params(d=d, omega_j=1.0, seed=21, noise="local")
    f = np.asarray(inputs.poisson_counts(dims, rho * lat.w, seed=21), dtype=np.float64)
    f = oracle.run(f, p, 40)
    rho_eq = f.sum() / N
    ks = np.array([[1, 0], [0, 1], [2, 1], [3, 2], [1, 4]])
    nlag, steps = 4, 3000
    res = oracle.correlate(f, p, steps, ks, 1, nlag, t0=40)
    n = res["nsamples"]
    S = res["sij"] / n / (N * rho_eq * np.sqrt(np.outer(lat.w, lat.w)))[None]
    # each diagonal entry is a mean of |f_i(k)|^2 with relative sd ~ 1 per
    # (nearly independent) sample; averaged over the k-list
    diag = np.array([np.real(np.diag(S[j])) for j in range(len(ks))])
    assert np.abs(diag.mean(axis=0) - 1).max() < 0.06
    off = np.array([S[j][~np.eye(lat.Q, dtype=bool)] for j in range(len(ks))])
    assert np.abs(off.mean(axis=0)).max() < 0.06
    for j, k in enumerate(ks):
        lam = cf.ftcs_factor(lat.theta, k, dims)
        c0 = res["ct"][j, 0].real / n
        for l in range(1, nlag):
            ratio = (res["ct"][j, l].real / (n - l)) / c0
            assert abs(ratio - lam ** l) < 0.08
