"""Pins of the oracle's statistics and of its stationary behaviour:
brute-force covariance on a few sites, the paper's Table I, flat S(k)."""

import os

import numpy as np
import pytest

import oracle
from paper_1606_07801_amd import inputs
from tests import closed_forms as cf


def _read_table1(golden_dir):
    out, cur = {}, None
    with open(os.path.join(golden_dir, "table1_dij.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("L "):
                cur = int(line.split()[1])
                out[cur] = []
            else:
                out[cur].append([float(x) for x in line.split()])
    return {k: np.array(v) for k, v in out.items()}


def test_lattice_sums_brute_force():
    gen = np.random.default_rng(1)
    f = gen.normal(1.0, 2.0, size=(5, 3, 4))
    f[2, 1, 1] = np.nan
    s = oracle.lattice_sums(f)
    Q = 5
    tot = 0.0
    ff = np.zeros((Q, Q))
    pos = 0.0
    neg = 0
    r2 = 0.0
    for y in range(3):
        for x in range(4):
            rho = sum(f[i, y, x] for i in range(Q))
            tot += rho
            r2 += rho * rho
            pos += max(rho, 0.0) if rho == rho else np.nan
            neg += int(rho < 0)
            for i in range(Q):
                for j in range(Q):
                    ff[i, j] += f[i, y, x] * f[j, y, x]
    assert s["nonfinite"] == 1 and s["nsite"] == 12
    g = f.copy()
    g[2, 1, 1] = 0.0
    s2 = oracle.lattice_sums(g)
    assert s2["nonfinite"] == 0
    rho = g.sum(axis=0)
    assert abs(s2["mass"] - rho.sum()) < 1e-12
    assert abs(s2["sum_rho2"] - (rho ** 2).sum()) < 1e-12
    assert s2["n_negative"] == int((rho < 0).sum())
    assert abs(s2["sum_rho_pos"] - np.maximum(rho, 0).sum()) < 1e-12
    ff2 = np.einsum("iyx,jyx->ij", g, g)
    assert np.abs(s2["sum_ff"] - ff2).max() < 1e-12


@pytest.mark.parametrize("shape", [(17,), (6, 10), (4, 5, 6)])
def test_structure_factor_direct_fft_parseval(shape):
    gen = np.random.default_rng(2)
    rho = gen.normal(3.0, 1.0, size=shape)
    d = rho.ndim
    L = shape[::-1]
    ks = np.array(np.meshgrid(*[np.arange(n) for n in L], indexing="ij")).reshape(d, -1).T
    a = oracle.structure_factor(rho, ks)
    b = oracle.structure_factor(rho, ks, method="fft")
    assert np.abs(a - b).max() < 1e-10 * a.max()
    # Parseval: sum_k |rho_k|^2 = N sum_x rho^2  ->  sum_k S(k) = sum_x rho^2
    assert abs(a.sum() - (rho ** 2).sum()) < 1e-9 * a.sum()
    # k = 0 is M^2 / N; k and -k agree for a real field
    assert abs(a[0] - rho.sum() ** 2 / rho.size) < 1e-12 * a[0]
    b2 = oracle.structure_factor(rho, -ks)
    assert np.abs(a - b2).max() < 1e-10 * a.max()


def _linear_step_matrix(lat, p, shape):
    """Noise-off step of the oracle as a matrix, column by column."""
    Q = lat.Q
    n = Q * int(np.prod(shape))
    A = np.empty((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        A[:, c] = oracle.step(e.reshape((Q,) + shape), lat, p, 0).ravel()
    return A


def test_brute_force_stationary_covariance_3x3(golden_dir):
    # Few-site brute force: iterate C <- A C A^T + Q_noise with the oracle's
    # noise-off step as A and the paper's f-space noise covariance (placed on
    # each colliding site, then streamed).  The fixed point must be
    # rho (w_i delta_ij delta_xx' - w_i w_j / N), which gives Table I's 3x3 values.
    rho = 120.0
    shape = (3, 3)
    nsite = 9
    for om in (0.6, 1.0, 1.8):
        p = oracle.Params(d=2, omega_j=om, noise="off")
        lat = p.lattice()
        Q = lat.Q
        A = _linear_step_matrix(lat, p, shape)
        # streaming alone: the step with Lambda = 0 is not available, so take
        # it from the oracle's stream function on unit vectors
        n = Q * nsite
        Smat = np.empty((n, n))
        for c in range(n):
            e = np.zeros(n)
            e[c] = 1.0
            Smat[:, c] = oracle.stream(e.reshape((Q,) + shape), lat).ravel()
        Lam = cf.lambda_f(lat.m, lat.n, p.omegas(lat))
        Qf = cf.fspace_noise_cov(lat.w, Lam, rho)
        # layout of the flat state: population-major (i, y, x)
        Qbig = np.kron(Qf, np.eye(nsite))
        Qs = Smat @ Qbig @ Smat.T
        C = np.zeros((n, n))
        for _ in range(400):
            C = A @ C @ A.T + Qs
        w = lat.w
        C_th = rho * (np.kron(np.diag(w), np.eye(nsite)) - np.kron(np.outer(w, w), np.ones((nsite, nsite))) / nsite)
        assert np.abs(C - C_th).max() < 1e-9 * rho
        # d_ij at one site
        dij = np.empty((Q, Q))
        for i in range(Q):
            for j in range(Q):
                dij[i, j] = C[i * nsite, j * nsite] / (rho * np.sqrt(w[i] * w[j]))
        assert np.abs(dij - cf.stationary_dij(w, nsite)).max() < 1e-10
    table = _read_table1(golden_dir)
    assert np.abs(table[3] - cf.stationary_dij(lat.w, 9)).max() < 1.5e-3


def test_closed_form_dij_matches_table1_all_sizes(golden_dir):
    table = _read_table1(golden_dir)
    w = oracle.make_lattice(2).w
    tol = {3: 1.5e-3, 10: 3e-4, 100: 4e-5}
    for L, t in table.items():
        assert np.abs(t - cf.stationary_dij(w, L * L)).max() < tol[L]


def test_monte_carlo_dij_3x3_reproduces_table1(golden_dir):
    # The oracle's own noisy trajectory, 3x3, rho^eq = 120, all rates 1,
    # local noise (Table I's setting, Gaussian instead of flat law: only the
    # variance enters d_ij).  The covariance is taken about the sample mean,
    # which removes the large linear terms of the raw estimator (dijexp)
    # without changing its expectation beyond O(1/samples).
    lat = oracle.make_lattice(2)
    rho = 120.0
    p = oracle.Params(d=2, omega_j=1.0, seed=2024, noise="local")
    f = inputs.outer(lat.w, np.full((3, 3), rho))
    for t in range(20):
        f = oracle.step(f, lat, p, t)
    snaps = []
    for t in range(20, 12020):
        f = oracle.step(f, lat, p, t)
        snaps.append(f.reshape(5, -1).copy())
    g = np.concatenate(snaps, axis=1)
    cov = np.cov(g)
    dij = cov / (rho * np.sqrt(np.outer(lat.w, lat.w)))
    table = _read_table1(golden_dir)[3]
    assert np.abs(dij - cf.stationary_dij(lat.w, 9)).max() < 0.02
    assert np.abs(dij - table).max() < 0.02
    # the finite-size deficit of the rest population is resolved
    assert dij[0, 0] < 0.985
    assert np.all(dij[~np.eye(5, dtype=bool)] < 0)


def _mc_structure_factor(d, dims, rho, noise, steps, seeds=(7, 8), burn=60):
    """S(k) for k = 1 .. L/2 along x, all rates one, averaged over steps and
    independent seeds; with its one-sigma error from the exact AR(1)
    correlation of a density mode at unit rates (gain lambda(k) per step)."""
    lat = oracle.make_lattice(d)
    L = dims[0]
    ks = np.array([[k] + [0] * (d - 1) for k in range(1, L // 2 + 1)])
    S = np.zeros(len(ks))
    pos = var = 0.0
    n = 0
    rho_eq = None
    for seed in seeds:
        p = oracle.Params(d=d, omega_j=1.0, seed=seed, noise=noise)
        f = inputs.poisson_counts(dims, rho * lat.w, seed=seed)
        rho_eq = f.sum() / f[0].size if rho_eq is None else rho_eq
        f *= rho_eq / (f.sum() / f[0].size)
        for t in range(burn + steps):
            f = oracle.step(f, lat, p, t, rho_eq=rho_eq)
            if t >= burn:
                r = f.sum(axis=0)
                S += oracle.structure_factor(r, ks, method="fft")
                pos += np.maximum(r, 0).mean()
                var += r.var()
                n += 1
    lam = np.array([cf.ftcs_factor(lat.theta, k, dims) for k in ks])
    rel_sigma = np.sqrt((1 + lam ** 2) / ((1 - lam ** 2) * n))
    return S / n, rel_sigma, pos / n, var / n, rho_eq


def test_flat_structure_factor_mean_density_10():
    S, sig, pos, var, rho_eq = _mc_structure_factor(1, (32,), 10.0, "local", 4000)
    z = (S / rho_eq - 1) / sig
    assert np.abs(z).max() < 4.5
    assert np.mean(z ** 2) < 2.5
    # equal-time density variance equals the mean: var = S (1 - 1/N)
    assert abs(var / (rho_eq * (1 - 1 / 32)) - 1) < 0.03


def test_flat_structure_factor_low_density_global():
    # global noise: S(k != 0) = rho^eq at any density, even rho = 0.1
    S, sig, pos, var, rho_eq = _mc_structure_factor(1, (32,), 0.1, "global", 4000)
    z = (S / rho_eq - 1) / sig
    assert np.abs(z).max() < 4.5
    assert np.mean(z ** 2) < 2.5
    assert abs(var / (rho_eq * (1 - 1 / 32)) - 1) < 0.04


def test_flat_structure_factor_low_density_local():
    # local noise with the clamp: S(k != 0) = <max(rho, 0)> (exceeds rho^eq at
    # low density, the direction the paper reports), still flat in k
    S, sig, pos, var, rho_eq = _mc_structure_factor(1, (32,), 0.1, "local", 4000)
    z = (S / pos - 1) / (1.5 * sig)
    assert np.abs(z).max() < 4.5
    assert np.mean(z ** 2) < 2.5
    assert pos > 1.3 * rho_eq
    assert abs(var / (pos * (1 - 1 / 32)) - 1) < 0.05


def test_flat_structure_factor_d2q5():
    S, sig, pos, var, rho_eq = _mc_structure_factor(2, (16, 8), 10.0, "local", 2500)
    z = (S / rho_eq - 1) / sig
    assert np.abs(z).max() < 4.5
    assert abs(var / (rho_eq * (1 - 1 / 128)) - 1) < 0.03


def test_poisson_initial_counts_table2(golden_dir):
    # Appendix eqs. (Poisson2), (f3): the Poisson rows of Table II, and the
    # generator's counts reproduce them.
    rows = {}
    with open(os.path.join(golden_dir, "table2_moments.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                r, kind, a, b, c = line.split()
                rows[(int(r), kind)] = (float(a), float(b), float(c))
    w1 = oracle.make_lattice(2).w[1]
    for r in (30, 1):
        mom = cf.poisson_moments(r * w1)
        tab = rows[(r, "poisson")]
        assert abs(mom[0] - tab[0]) <= 1e-3 * max(1, tab[0])
        assert abs(mom[1] - tab[1]) <= 1e-3 * max(1, tab[1])
        assert abs(mom[2] - tab[2]) <= 2e-3 * max(1, tab[2])
        counts = inputs.poisson_counts((400, 400), [r * w1], seed=r)[0]
        emp = (counts.mean(), (counts ** 2).mean(), (counts ** 3).mean())
        for e, m in zip(emp, mom):
            assert abs(e / m - 1) < 0.02


@pytest.mark.parametrize("shape", [(7,), (4, 6), (3, 4, 5)])
def test_profile_brute_force(shape):
    # sums of rho and rho^2 over the sites of each coordinate, by explicit loops
    gen = np.random.default_rng(11)
    d = len(shape)
    Q = 2 * d + 1
    f = gen.normal(1.0, 2.0, size=(Q,) + tuple(reversed(shape)))
    rho = f.sum(axis=0)
    for axis in range(d):
        s, s2 = oracle.profile(f, axis)
        ref, ref2 = np.zeros(shape[axis]), np.zeros(shape[axis])
        for idx in np.ndindex(*rho.shape):
            c = idx[d - 1 - axis]              # array index order is (.., y, x)
            ref[c] += rho[idx]
            ref2[c] += rho[idx] ** 2
        assert np.allclose(s, ref, rtol=1e-13, atol=1e-12)
        assert np.allclose(s2, ref2, rtol=1e-13, atol=1e-12)
