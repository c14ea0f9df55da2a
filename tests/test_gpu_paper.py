"""The paper's equilibrium measurements reproduced on the GPU path, with the
paper's own noise law (flat, Sec. IV): Table I (finite-size d_ij on 3x3, 10x10, 100x100),
Table II (low-density population moments) with the histograms of Fig. 4, Fig. 1
(the mean populations over density and relaxation time) and Fig. 3 (the
population correlators over density, local against global noise).  The
Table II noise rows are the paper's Monte Carlo values on an unstated
lattice size and run length, so they are compared loosely; with global noise
the second moment is checked against the Poisson value that the linear update
fixes exactly."""

import os

import numpy as np
import pytest

from paper_1606_07801_amd import experiments
from tests import closed_forms as cf

pytestmark = pytest.mark.gpu


def _table(golden_dir, name):
    return open(os.path.join(golden_dir, name)).read().splitlines()


def test_table1_3x3_dij(golden_dir):
    rows = _table(golden_dir, "table1_dij.txt")
    i = rows.index("L 3")
    table = np.array([[float(x) for x in r.split()] for r in rows[i + 1:i + 6]])
    d = experiments.dij(3, rho=120.0, steps=300_000, law="uniform", noise="local", seed=11)
    w = np.array([1 / 3] + [1 / 6] * 4)
    closed = cf.stationary_dij(w, 9)
    print("[table1] d_ij 3x3 (GPU, uniform law, local noise):\n", np.round(d, 5))
    assert np.abs(d - closed).max() < 0.01
    assert np.abs(d - table).max() < 0.01
    assert d[0, 0] < 0.975 and np.all(d[~np.eye(5, dtype=bool)] < 0)


@pytest.mark.parametrize("side", [10, 100])
def test_table1_larger_lattices_dij(golden_dir, side):
    # Table I's 10x10 and 100x100 blocks with the paper's 1.7e6 iterations.
    # The sample covariance of N T site samples has a standard error of about
    # sqrt((1 + d_ij^2) / (N T)) in d_ij: 1.1e-4 / 7.7e-5 (diagonal / off)
    # at 10x10 and 1.1e-5 / 7.7e-6 at 100x100, against finite-size terms
    # -sqrt(w_i w_j) / N of 1.7e-3 and 1.7e-5.
    rows = _table(golden_dir, "table1_dij.txt")
    i = rows.index(f"L {side}")
    table = np.array([[float(x) for x in r.split()] for r in rows[i + 1:i + 6]])
    N, T = side * side, 1_700_000
    d = experiments.dij(side, rho=120.0, steps=T, law="uniform", noise="local", seed=13)
    w = np.array([1 / 3] + [1 / 6] * 4)
    closed = cf.stationary_dij(w, N)
    se = np.sqrt((1 + closed ** 2) / (N * T))
    z = (d - closed) / se
    off = ~np.eye(5, dtype=bool)
    print(f"[table1] L={side}: max |d - closed| {np.abs(d - closed).max():.2e} (max |z| {np.abs(z).max():.1f}), "
          f"max |d - paper| {np.abs(d - table).max():.2e}; mean off-diagonal {d[off].mean():.3e} "
          f"(closed {closed[off].mean():.3e}, paper {table[off].mean():.3e})", flush=True)
    assert np.abs(z).max() < 6.0
    assert np.abs(d - table).max() < 8 * se.max()
    # the finite-size anticorrelation is resolved: the mean off-diagonal entry
    # lies below zero by more than six of its standard errors (bounded by the
    # largest single-entry error over sqrt(20), entries nearly independent)
    assert d[off].mean() < -6 * se[off].max() / np.sqrt(20)


@pytest.mark.parametrize("rho", [30.0, 1.0])
@pytest.mark.parametrize("noise", ["local", "global"])
def test_table2_low_density_moments(golden_dir, rho, noise):
    rows = {}
    for line in _table(golden_dir, "table2_moments.txt"):
        if line.strip() and not line.startswith("#"):
            r, kind, a, b, c = line.split()
            rows[(float(r), kind)] = (float(a), float(b))
    w, mf, mff = experiments.population_moments(128, rho, steps=3000, burn=300, noise=noise, law="uniform",
                                                seed=5)
    f1, f11 = mf[1:].mean(), np.mean([mff[i, i] for i in range(1, 5)])
    paper = rows[(rho, noise)]
    poisson = rows[(rho, "poisson")]
    print(f"[table2] rho={rho} {noise}: <f1>={f1:.5f} <f1^2>={f11:.5f}  paper {paper}  Poisson {poisson}")
    assert abs(f1 / (rho / 6) - 1) < 2e-3          # mass: <f_1> = rho w_1 exactly in expectation
    if noise == "global":
        # Global noise makes the update linear in f with additive noise, so the
        # second moment is the Poisson one of eq. (ffluct) at every density.
        # The paper's rho = 1 global row (first moment 0.1711) cannot come from
        # a mass-conserving linear update and is not reproduced; at rho = 30 it
        # agrees with the Poisson value to 0.1 %.
        assert abs(f11 / poisson[1] - 1) < 3e-3
        if rho >= 30:
            assert abs(f11 / paper[1] - 1) < 0.01
    else:
        # local noise: the paper's low-density excess over Poisson is reproduced
        tol = 0.01 if rho >= 30 else 0.03
        assert abs(f11 / paper[1] - 1) < tol
        if rho < 30:
            assert f11 > poisson[1] * 1.03


def _mean_se(x):
    """Batch means (axis 0: batches) -> mean and standard error."""
    x = np.asarray(x)
    return x.mean(axis=0), x.std(axis=0, ddof=1) / np.sqrt(x.shape[0])


def test_fig1_equilibrium_mean_over_density_and_tau():
    # Fig. 1: the space-time mean of every population equals f_i^eq = w_i rho
    # at all densities and relaxation times (local noise, flat law, theta = 1/3)
    dens = [0.5, 2.0, 10.0, 100.0]
    worst = 0.0
    for tau in (0.6, 1.0, 2.0):
        w, r = experiments.density_sweep(dens, noise="local", omega=1.0 / tau, steps=80_000, batches=20)
        for j, rho in enumerate(dens):
            m, se = _mean_se(r["f"][j])
            z = (m - w * rho) / np.maximum(se, 1e-12)
            rel = np.abs(m / (w * rho) - 1)
            worst = max(worst, np.abs(z).max())
            print(f"[fig1] tau={tau} rho={rho}: max |<f_i>/f_eq - 1| = {rel.max():.2e} (max |z| {np.abs(z).max():.1f})",
                  flush=True)
            assert rel.max() < 5e-3
    assert worst < 7.0


def test_fig3_low_density_correlators():
    # Fig. 3: <f_i f_i> over the Poisson prediction f_eq^2 + f_eq, against the
    # mean density.  Global noise: the update is linear with additive noise,
    # so the site variance is exactly rho (w_i - w_i^2 / N) and the ratio is 1
    # at every density.  Local noise: the clamp at rho = 0 makes the noise
    # density <max(rho, 0)> > rho, the site variance <rho+> (w_i - w_i^2 / N)
    # (the same linear response), so the fluctuations grow at low density --
    # the paper's observation -- by a percent near rho = 3.
    dens = [0.5, 1.0, 2.0, 3.0, 5.0, 7.0, 10.0, 30.0]
    N = 32 * 32
    ratio = {}
    for noise in ("global", "local"):
        w, r = experiments.density_sweep(dens, noise=noise, steps=200_000, batches=20)
        ratio[noise] = []
        for j, rho in enumerate(dens):
            f, _ = _mean_se(r["f"][j])
            ff_b = r["ff"][j]
            pred = (w * rho) ** 2 + w * rho
            q, q_se = _mean_se(ff_b / pred[None, :])
            pos, _ = _mean_se(r["pos"][j])
            neg, _ = _mean_se(r["neg"][j])
            ratio[noise].append(q)
            # the exact stationary variance for either noise: rho_n (w_i - w_i^2 / N),
            # rho_n = rho (global) or <rho+> (local)
            rho_n = rho if noise == "global" else pos
            var_pred = rho_n * (w - w ** 2 / N)
            var, var_se = _mean_se(ff_b - r["f"][j] ** 2)
            zv = (var - var_pred) / np.maximum(var_se, 1e-15)
            print(f"[fig3] {noise:6s} rho={rho:5.1f}: <f_i f_i>/pred - 1 = {np.round(q - 1, 4)} "
                  f"(se {q_se.max():.1e}); <rho+>/rho - 1 = {pos / rho - 1:.4f}; negative sites {neg:.4f}; "
                  f"variance z {np.abs(zv).max():.1f}", flush=True)
            assert np.abs(zv).max() < 6.0
            if noise == "global":
                assert np.abs(q - 1).max() < max(6 * q_se.max(), 2e-3)
        ratio[noise] = np.array(ratio[noise])
    loc = ratio["local"][:, 1:].mean(axis=1)       # moving populations
    glo = ratio["global"][:, 1:].mean(axis=1)
    # local noise: fluctuations above the prediction at low density, rising as
    # the density falls, with the 1 % excess crossed between rho = 2 and 3 (the
    # paper places that threshold near rho = 3); global noise stays at 1
    print(f"[fig3] moving populations, local: {np.round(loc - 1, 4)}; global: {np.round(glo - 1, 4)}", flush=True)
    assert np.all(np.diff(loc) < 0.002)
    assert loc[0] > 1.02 and abs(loc[-1] - 1) < 0.002
    assert loc[dens.index(2.0)] - 1 > 0.01 > loc[dens.index(3.0)] - 1


@pytest.mark.parametrize("rho", [30.0, 1.0])
def test_table2_third_moment_and_fig4_histogram(golden_dir, rho):
    # Table II's third column and the histograms of Fig. 4 (f_1 with a bin of
    # one particle at rho = 30 and a tenth at rho = 1).
    rows = {}
    for line in _table(golden_dir, "table2_moments.txt"):
        if line.strip() and not line.startswith("#"):
            r, kind, a, b, c = line.split()
            rows[(float(r), kind)] = (float(a), float(b), float(c))
    side, N = 128, 128 * 128
    step = 1.0 if rho == 30.0 else 0.1
    lo, hi = (-12.0, 60.0) if rho == 30.0 else (-1.0, 2.0)
    edges = np.round(np.arange(lo, hi + step / 2, step), 10)
    out = {}
    for noise in ("global", "local"):
        r = experiments.population_distribution(side, rho, steps=3000, edges=edges, noise=noise, law="uniform",
                                                seed=7)
        m, se = _mean_se(r["m"])
        assert int(r["hist"].sum()) + r["under"] + r["over"] == r["samples"]
        out[noise] = (m, se, r)
        i0 = int(np.searchsorted(edges, 0.0, side="right")) - 1      # the bin starting at 0
        near = r["hist"][max(i0 - 3, 0):i0 + 3] / r["samples"] / step
        print(f"[table2/fig4] rho={rho} {noise}: <f1>={m[0]:.5f} <f1^2>={m[1]:.5f} <f1^3>={m[2]:.5f} "
              f"(se {se[2]:.1e}); paper {rows[(rho, noise)]}; Poisson {rows[(rho, 'poisson')]}; "
              f"f1 < 0: {(r['hist'][:i0].sum() + r['under']) / r['samples']:.4f}; f1 == 0: {r['zero']}; "
              f"density near 0 {np.round(near, 3)}", flush=True)
    # Global noise: a linear update with symmetric noise independent of the
    # state, from the deterministic start f = w rho, keeps the third cumulant
    # at zero, so <f^3> = mu^3 + 3 mu var with mu = w_1 rho and the exact
    # variance rho (w_1 - w_1^2 / N).
    w1 = 1.0 / 6.0
    mu, var = w1 * rho, rho * (w1 - w1 * w1 / N)
    m, se, _ = out["global"]
    z = (m - np.array([mu, mu * mu + var, mu ** 3 + 3 * mu * var])) / se
    print(f"[table2] global closed form <f1^3> = {mu ** 3 + 3 * mu * var:.5f}; z = {np.round(z, 2)}", flush=True)
    assert np.abs(z).max() < 6.0
    if rho == 30.0:
        assert abs(m[2] / rows[(rho, "global")][2] - 1) < 0.01      # printed 200
    # Local noise: the state-dependent amplitude gives a positive third
    # cumulant, so <f^3> lies above the global value (the paper's trend).
    ml, sel, rl = out["local"]
    assert ml[2] > m[2] + 6 * max(sel[2], se[2])
    assert abs(ml[2] / rows[(rho, "local")][2] - 1) < (0.01 if rho == 30.0 else 0.03)   # 202, 0.164
    if rho == 1.0:
        # Fig. 4b's peak at zero: with local noise a site whose density is
        # near or below zero gets little or no noise, so f_1 = rho / 6 piles
        # up just below zero (the bin [-0.1, 0) holds twice its neighbours'
        # density).  Global noise has a fixed amplitude and no such peak.
        i0 = int(np.searchsorted(edges, 0.0, side="right")) - 1
        hl, hg = rl["hist"], out["global"][2]["hist"]
        assert hl[i0 - 1] > 1.5 * max(hl[i0 - 2], hl[i0])
        assert hg[i0 - 1] < 1.05 * max(hg[i0 - 2], hg[i0])
