"""Pins of the oracle's time step against closed forms, special cases and
invariants that the paper and the mathematics fix."""

import numpy as np
import pytest

import oracle
from paper_1606_07801_amd import inputs
from tests import closed_forms as cf

DIMS = {1: (40,), 2: (24, 14), 3: (10, 8, 6)}


def _lat(d, theta=None):
    return oracle.make_lattice(d, theta)


def _random_state(d, rho=10.0, seed=0, dims=None):
    lat = _lat(d)
    dims = dims or DIMS[d]
    return inputs.poisson_counts(dims, rho * lat.w, seed=seed)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("noise", ["local", "global"])
def test_mass_conservation(d, noise):
    # Sec. IV: sum_x sum_i f_i is constant; the noise has zero component on
    # the conserved moment (eq. xiglobal / xilocal).
    f = _random_state(d, rho=10.0, seed=d)
    p = oracle.Params(d=d, omega_j=1.3, omega_n=0.7, omega_s=1.6, seed=4, noise=noise)
    m0 = f.sum()
    g = oracle.run(f, p, 30)
    # exact in real arithmetic; in FP64 each site-step may add a rounding
    # error of a few ulp of rho, with a systematic sign at worst
    bound = 4 * f.shape[0] * np.finfo(float).eps * np.abs(f.sum(axis=0)).sum() * 30
    assert abs(g.sum() - m0) < bound
    assert np.abs(g - f).max() > 0.1          # the state did change


@pytest.mark.parametrize("d", [1, 2, 3])
def test_noise_has_no_mass_at_each_site(d):
    lat = _lat(d)
    f = _random_state(d, rho=7.0, seed=1)
    Q = lat.Q
    flat = f.reshape(Q, -1)
    idx = np.arange(flat.shape[1], dtype=np.uint64)
    p = oracle.Params(d=d, omega_j=0.8, seed=11)
    fs = oracle.collide(flat, idx, lat, p, 5)
    assert np.abs(fs.sum(axis=0) - flat.sum(axis=0)).max() < 1e-12


@pytest.mark.parametrize("d", [1, 2, 3])
def test_unit_rate_is_explicit_diffusion_scheme(d):
    # Sec. IV, equilibrium dynamics: with all rates one and no noise,
    # rho(x, t+1) = sum_i w_i rho(x - v_i, t), and every population leaves
    # the collision at f_i* = w_i rho.
    lat = _lat(d)
    f = _random_state(d, rho=10.0, seed=3)
    p = oracle.Params(d=d, omega_j=1.0, noise="off")
    g = oracle.step(f, lat, p, 0)
    rho = f.sum(axis=0)
    expect = np.zeros_like(rho)
    for i in range(lat.Q):
        shift = tuple(int(lat.v[i, a]) for a in range(d))
        expect += lat.w[i] * np.roll(rho, shift, axis=tuple(-1 - a for a in range(d)))
    assert np.abs(g.sum(axis=0) - expect).max() < 1e-12
    for i in range(lat.Q):
        shift = tuple(int(lat.v[i, a]) for a in range(d))
        assert np.abs(g[i] - lat.w[i] * np.roll(rho, shift, axis=tuple(-1 - a for a in range(d)))).max() < 1e-12


def _mode_amplitude(rho, k):
    d = rho.ndim
    L = rho.shape[::-1]
    grids = np.meshgrid(*[np.arange(n) for n in rho.shape], indexing="ij")[::-1]
    ph = sum(2 * np.pi * k[a] * grids[a] / L[a] for a in range(d))
    return np.sum(rho * np.exp(-1j * ph))


@pytest.mark.parametrize("d,dims,k", [(1, (32,), (3,)), (2, (16, 12), (2, 1)), (3, (8, 6, 10), (1, 2, 3))])
@pytest.mark.parametrize("omegas", [(1.0, 0, 0), (0.6, 0, 0), (1.8, 0, 0), (1.2, 0.5, 1.7)])
def test_noise_off_mode_decay_matches_transfer_matrix(d, dims, k, omegas):
    # Noise-off evolution of a single density mode: the oracle's trajectory
    # against the product of one-step Fourier transfer matrices.
    lat = _lat(d)
    p = oracle.Params(d=d, omega_j=omegas[0], omega_n=omegas[1], omega_s=omegas[2], noise="off")
    L = dims
    # f_i = w_i * cos(k.x) real mode: a_k(0) = N/2
    shape = inputs.array_shape(dims)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")[::-1]
    ph = sum(2 * np.pi * k[a] * grids[a] / L[a] for a in range(d))
    rho0 = 10.0 + np.cos(ph)
    f = inputs.outer(lat.w, rho0)
    t = 40
    g = oracle.run(f, p, t)
    a_t = _mode_amplitude(g.sum(axis=0), k)
    a_0 = _mode_amplitude(rho0, k)
    Lam = cf.lambda_f(lat.m, lat.n, p.omegas(lat))
    gain = cf.density_gain(lat.w, lat.v, k, L, Lam, t)
    assert abs(a_t - gain * a_0) < 1e-10 * abs(a_0)
    # the k = 0 mode is the mass and does not change
    assert abs(_mode_amplitude(g.sum(axis=0), (0,) * d) - rho0.sum()) < 1e-9


@pytest.mark.parametrize("d", [1, 2, 3])
def test_unit_rate_factor_is_the_papers_dispersion(d):
    # all rates one: the one-step gain of a density mode equals
    # 1 - theta (d - sum cos(2 pi k_a / L_a))
    lat = _lat(d)
    L = (16, 12, 10)[:d]
    Lam = cf.lambda_f(lat.m, lat.n, np.ones(lat.Q))
    for k in [(1, 0, 0), (3, 2, 1), (8, 6, 5)]:
        k = k[:d]
        g1 = cf.density_gain(lat.w, lat.v, k, L, Lam, 1)
        assert abs(g1 - cf.ftcs_factor(lat.theta, k, L)) < 1e-14


@pytest.mark.parametrize("omega", [0.6, 1.0, 1.5])
def test_small_k_decay_gives_diffusion_constant(omega):
    # Sec. III: D = (tau^j - 1/2) theta; a long-wavelength mode decays as exp(-D k^2 t).
    lat = _lat(1)
    L = (4096,)
    Lam = cf.lambda_f(lat.m, lat.n, np.full(lat.Q, omega))
    T = cf.mode_matrix(lat.w, lat.v, (1,), L, Lam)
    ev = np.linalg.eigvals(T)
    slow = ev[np.argmax(np.abs(ev))]
    kk = 2 * np.pi / L[0]
    D = (1.0 / omega - 0.5) * lat.theta
    assert abs(-np.log(abs(slow)) / (D * kk * kk) - 1.0) < 1e-3


def test_y_uniform_d2q5_equals_d1q3():
    # Reduction: with one relaxation rate and no noise a D2Q5 field that is
    # uniform in y evolves like D1Q3 at the same theta (the +-y populations do
    # not move the field and add to the rest population).
    th = 0.3
    L = 48
    x = np.arange(L)
    rho = 5.0 + np.sin(2 * np.pi * 3 * x / L) + 0.5 * np.cos(2 * np.pi * 7 * x / L)
    l1, l2, l3 = _lat(1, th), _lat(2, th), _lat(3, th)
    f1 = inputs.outer(l1.w, rho)
    f2 = inputs.outer(l2.w, np.broadcast_to(rho, (5, L)).copy())
    f3 = inputs.outer(l3.w, np.broadcast_to(rho, (3, 4, L)).copy())
    for om in (0.7, 1.0, 1.9):
        g1 = oracle.run(f1, oracle.Params(d=1, theta=th, omega_j=om, noise="off"), 25)
        g2 = oracle.run(f2, oracle.Params(d=2, theta=th, omega_j=om, noise="off"), 25)
        g3 = oracle.run(f3, oracle.Params(d=3, theta=th, omega_j=om, noise="off"), 25)
        assert np.abs(g2.sum(axis=0) - g1.sum(axis=0)[None, :]).max() < 1e-12
        assert np.abs(g3.sum(axis=0) - g1.sum(axis=0)[None, None, :]).max() < 1e-12


def _noise_samples(d, p, rho, nsite=200_000, t=2):
    lat = _lat(d, p.theta)
    f = np.repeat((lat.w * rho)[:, None], nsite, axis=1)
    idx = np.arange(nsite, dtype=np.uint64)
    with_noise = oracle.collide(f, idx, lat, p, t, rho_eq=rho)
    q = oracle.Params(**{**p.__dict__, "noise": "off"})
    return lat, with_noise - oracle.collide(f, idx, lat, q, t)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("law", ["gauss", "uniform"])
@pytest.mark.parametrize("om", [(1.0, 0, 0), (1.4, 0.6, 1.9)])
def test_noise_covariance_is_the_papers_fspace_law(d, law, om):
    # Sec. II: <xi_i xi_j> in f-space for the collision matrix Lambda, and
    # diagonal form rho (2 tau^a - 1)/(tau^a)^2 in moment space.
    rho = 6.0
    p = oracle.Params(d=d, omega_j=om[0], omega_n=om[1], omega_s=om[2], seed=17, law=law)
    lat, xi = _noise_samples(d, p, rho)
    Lam = cf.lambda_f(lat.m, lat.n, p.omegas(lat))
    C_th = cf.fspace_noise_cov(lat.w, Lam, rho)
    C = np.cov(xi)
    scale = np.sqrt(np.outer(np.diag(C_th), np.diag(C_th)))
    assert np.abs(C - C_th).max() < 0.02 * scale.max()
    # moment space: diagonal with variance rho * omega (2 - omega), zero on rho
    Mxi = lat.m @ xi
    var = Mxi.var(axis=1)
    oms = p.omegas(lat)
    assert var[0] < 1e-20
    assert np.abs(var[1:] / (rho * oms[1:] * (2 - oms[1:])) - 1).max() < 0.02
    # law: Gaussian kurtosis 3, flat law 9/5
    kurt = np.mean(Mxi[1:] ** 4, axis=1) / var[1:] ** 2
    target = 3.0 if law == "gauss" else 1.8
    assert np.abs(kurt - target).max() < 0.1


def test_negative_density_suspends_local_noise_only():
    # Sec. IV: a negative density is treated as zero in the noise amplitude.
    lat = _lat(2)
    f = inputs.outer(lat.w, -np.ones((6, 7)) * 0.3)
    f[1] += 0.001 * np.arange(42).reshape(6, 7)
    p = oracle.Params(d=2, omega_j=1.1, seed=3, noise="local")
    off = oracle.Params(d=2, omega_j=1.1, seed=3, noise="off")
    a = oracle.step(f, lat, p, 0)
    b = oracle.step(f, lat, off, 0)
    assert np.array_equal(a, b)
    glob = oracle.Params(d=2, omega_j=1.1, seed=3, noise="global")
    c = oracle.step(f, lat, glob, 0, rho_eq=2.0)
    assert np.abs(c - b).max() > 0.1


def test_global_noise_uses_mean_density():
    rho_eq = 3.0
    p = oracle.Params(d=2, omega_j=1.0, seed=8, noise="global")
    lat = _lat(2)
    nsite = 100_000
    # local densities far from rho_eq: the amplitude must not follow them
    f = np.repeat((lat.w * 50.0)[:, None], nsite, axis=1)
    idx = np.arange(nsite, dtype=np.uint64)
    xi = oracle.collide(f, idx, lat, p, 0, rho_eq=rho_eq) - oracle.collide(
        f, idx, lat, oracle.Params(d=2, omega_j=1.0, noise="off"), 0)
    var = (lat.m @ xi).var(axis=1)
    assert np.abs(var[1:] / rho_eq - 1).max() < 0.03


def test_step_sites_matches_full_step():
    for d in (1, 2, 3):
        lat = _lat(d)
        f = _random_state(d, rho=4.0, seed=9)
        p = oracle.Params(d=d, omega_j=1.3, seed=21)
        g = oracle.step(f, lat, p, 6)
        shape = f.shape[1:]
        L = shape[::-1]
        gen = np.random.default_rng(0)
        coords = np.stack([gen.integers(0, L[a], 50) for a in range(d)], axis=1)
        vals = oracle.step_sites(f, lat, p, 6, coords)
        for n, c in enumerate(coords):
            idx = tuple(int(c[a]) for a in reversed(range(d)))
            assert np.abs(g[(slice(None),) + idx] - vals[:, n]).max() < 1e-13


def test_noise_depends_on_seed_and_step():
    lat = _lat(1)
    f = _random_state(1, seed=2)
    a = oracle.step(f, lat, oracle.Params(d=1, seed=1), 0)
    b = oracle.step(f, lat, oracle.Params(d=1, seed=2), 0)
    c = oracle.step(f, lat, oracle.Params(d=1, seed=1), 1)
    assert np.abs(a - b).max() > 0.1 and np.abs(a - c).max() > 0.1
    # every bit of the 32-bit step word keys the noise
    for t in (1 << 16, 1 << 31):
        e = oracle.step(f, lat, oracle.Params(d=1, seed=1), t)
        assert np.abs(a - e).max() > 0.1


@pytest.mark.parametrize("d", [1, 2, 3])
def test_uniform_state_relaxes_each_class_at_its_rate(d):
    # A spatially uniform state is not changed by streaming, so one step is a
    # pure collision: with the noise off, the physical moments
    #   j_a = sum_i f_i v_ia,  traceless sum_i f_i (v_x^2 - v_y^2),
    #   trace excess sum_i f_i (|v|^2 - d theta)
    # relax by (1 - omega) of their class (Sec. II, diagonal Lambda^ab;
    # Sec. III, isotropy classes j, n, s).
    lat = _lat(d)
    oj, on, os_ = 0.35, 1.45, 1.85
    p = oracle.Params(d=d, omega_j=oj, omega_n=on, omega_s=os_, noise="off")
    gen = np.random.default_rng(d)
    f = np.ones((lat.Q,) + (3,) * d) * (lat.w + 0.2 * gen.random(lat.Q)).reshape((-1,) + (1,) * d)
    g = oracle.step(f, lat, p, 0)
    v = lat.v.astype(float)

    def mom(h, vec):
        return np.tensordot(vec, h[(slice(None),) + (0,) * d], axes=(0, 0))

    for a in range(d):
        assert abs(mom(g, v[:, a]) - (1 - oj) * mom(f, v[:, a])) < 1e-13
    v2 = (v ** 2).sum(axis=1)
    rho = mom(f, np.ones(lat.Q))
    tr_f = mom(f, v2) - d * lat.theta * rho
    tr_g = mom(g, v2) - d * lat.theta * rho
    assert abs(tr_g - (1 - os_) * tr_f) < 1e-13
    if d >= 2:
        tl = v[:, 0] ** 2 - v[:, 1] ** 2
        assert abs(mom(g, tl) - (1 - on) * mom(f, tl)) < 1e-13


def test_moment_a_takes_variate_a_minus_1():
    # Noise stream convention: moment a >= 1 takes variate a - 1 of
    # noise_draws (block (a-1) // 4, word (a-1) % 4).
    for d in (1, 2, 3):
        lat = _lat(d)
        p = oracle.Params(d=d, omega_j=1.0, seed=31)
        nsite = 4000
        f = np.repeat((lat.w * 9.0)[:, None], nsite, axis=1)
        idx = np.arange(nsite, dtype=np.uint64)
        xi = oracle.collide(f, idx, lat, p, 4) - oracle.collide(
            f, idx, lat, oracle.Params(d=d, omega_j=1.0, noise="off"), 4)
        z = oracle.noise_draws(lat, 31, 4, idx)
        M = lat.m @ xi
        for a in range(1, lat.Q):
            assert np.allclose(M[a], 3.0 * z[a - 1], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d,T", [(1, 7), (2, 5), (3, 3)])
def test_run_sites_matches_full_run(d, T):
    lat = _lat(d)
    dims = {1: (30,), 2: (16, 13), 3: (9, 8, 7)}[d]
    f = _random_state(d, rho=5.0, seed=4, dims=dims)
    for noise in ("local", "global"):
        p = oracle.Params(d=d, omega_j=1.4, omega_s=0.8, seed=13, noise=noise)
        rho_eq = f.sum() / f[0].size
        g = oracle.run(f, p, T, t0=11, rho_eq=rho_eq)
        gen = np.random.default_rng(1)
        coords = np.stack([gen.integers(0, dims[a], 25) for a in range(d)], axis=1)
        vals = oracle.run_sites(f, lat, p, 11, T, coords, rho_eq=rho_eq)
        for n, c in enumerate(coords):
            idx = tuple(int(c[a]) for a in reversed(range(d)))
            assert np.abs(g[(slice(None),) + idx] - vals[:, n]).max() < 1e-12


@pytest.mark.parametrize("d,T", [(1, 9), (2, 6), (3, 3)])
def test_run_box_matches_full_run(d, T):
    # a box that wraps around the periodic edge of every axis, and one larger
    # than the lattice along x (its window then repeats sites)
    lat = _lat(d)
    dims = {1: (30,), 2: (16, 13), 3: (9, 8, 7)}[d]
    f = _random_state(d, rho=5.0, seed=6, dims=dims)
    for noise in ("local", "global"):
        p = oracle.Params(d=d, omega_j=1.2, omega_n=1.7, seed=19, noise=noise)
        rho_eq = f.sum() / f[0].size
        g = oracle.run(f, p, T, t0=4, rho_eq=rho_eq)
        for origin, extent in (([dims[a] - 3 for a in range(d)], [5] * d),
                               ([1] + [0] * (d - 1), [dims[0] + 4] + [2] * (d - 1))):
            box = oracle.run_box(f, lat, p, 4, T, origin, extent, rho_eq=rho_eq)
            idx = np.ix_(*[(origin[a] + np.arange(extent[a])) % dims[a] for a in reversed(range(d))])
            assert box.shape == (lat.Q,) + tuple(reversed(extent))
            assert np.abs(box - g[(slice(None),) + idx]).max() < 1e-12


@pytest.mark.parametrize("d,T,H", [(1, 8, 5), (2, 6, 4), (2, 3, 3), (3, 3, 2)])
def test_run_box_light_cone_minimum(d, T, H):
    # brute force: the full-lattice trajectory's |rho| at every collision of
    # the last H steps, minimised over each box site's periodic L1 ball of
    # radius (steps left after that collision)
    lat = _lat(d)
    dims = {1: (30,), 2: (16, 13), 3: (9, 8, 7)}[d]
    f = inputs.gaussian_field(dims, 0.4, 1.0, seed=3)[None] * lat.w.reshape((-1,) + (1,) * d)
    p = oracle.Params(d=d, omega_j=1.0, seed=2)
    rhos, g = [], f
    for t in range(T):
        rhos.append(np.abs(g.sum(axis=0)))
        g = oracle.step(g, lat, p, t)
    origin, extent = [dims[a] - 2 for a in range(d)], [4] * d
    box, mr = oracle.run_box(f, lat, p, 0, T, origin, extent, horizon=H)
    assert np.abs(box - g[(slice(None),) + np.ix_(*[(origin[a] + np.arange(4)) % dims[a]
                                                     for a in reversed(range(d))])]).max() < 1e-12
    grids = np.meshgrid(*[np.arange(4)] * d, indexing="ij")   # box offsets, array order (.., x)
    for pos in zip(*[gi.ravel() for gi in grids]):
        x = [(origin[a] + pos[d - 1 - a]) % dims[a] for a in range(d)]
        best = np.inf
        for t in range(T - H, T):
            r = T - t
            for q in np.ndindex(*reversed(dims)):          # q in array order (.., y, x)
                dist = sum(min(abs(q[d - 1 - a] - x[a]), dims[a] - abs(q[d - 1 - a] - x[a])) for a in range(d))
                if dist <= r:
                    best = min(best, rhos[t][q])
        assert mr[pos] == best


def test_noise_off_front_follows_the_erf_solution():
    # Sec. IV, non-equilibrium dynamics: at unit rates (D = theta / 2) the
    # deterministic block profile of a y-uniform D2Q5 strip approaches the
    # continuum erf solution as the front widens
    lat = oracle.make_lattice(2)
    x = np.arange(100)
    rho0 = np.where((x >= 25) & (x < 75), 20.0, 120.0)
    f = lat.w[:, None, None] * rho0[None, None, :]
    p = oracle.Params(d=2, omega_j=1.0, noise="off")
    prev, errs = 0, []
    for t in (100, 400, 1600):
        f = oracle.run(f, p, t - prev, t0=prev)
        prev = t
        errs.append(np.abs(f.sum(axis=0)[0] - cf.front_profile(100, t, lat.theta / 2, 20.0, 120.0)).max())
    assert errs[0] < 0.05 and errs[1] < 0.01 and errs[2] < 0.005
    assert errs[2] < errs[1] < errs[0]
