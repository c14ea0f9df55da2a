"""Population correlators on the GPU path (Sec. IV: the Fourier test,
eqs. fkfk / FourierTest, and the equilibrium dynamics, eq. TimeCorrEqn):
element-wise parity with the oracle on the same seeded inputs, edge cases,
and the paper's two measurements -- S_ij(k) flat apart from k = 0 (Fig. 2)
and the density time correlator decaying with the explicit scheme's gain
(Fig. 7)."""

import numpy as np
import pytest

import oracle
from paper_1606_07801_amd import flb, inputs
from tests import closed_forms as cf
from tests.gpu_common import gpu_lattice, poisson_state

pytestmark = pytest.mark.gpu

KS = {
    1: [[0], [1], [-3], [17], [999], [1500], [500]],
    2: [[0, 0], [1, 0], [0, 1], [-2, 5], [150, 35], [299, 69], [7, -11], [400, 3], [13, 13]],
    3: [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 2, 3], [6, 5, 4], [11, 9, 8]],
}
CASES = [(1, (1000,)), (2, (300, 70)), (3, (12, 10, 9))]
TOL = {8: 1e-10, 4: 3e-5}


def _scale(f0):
    A = np.abs(np.asarray(f0, dtype=np.float64)).reshape(f0.shape[0], -1).sum(axis=1)
    return A


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("d,dims", CASES)
def test_amplitudes_match_oracle(d, dims, precision):
    dt = np.float32 if precision == 4 else np.float64
    f0 = poisson_state(d, dims, 10.0, seed=3).astype(dt)
    ks = np.array(KS[d])
    L = gpu_lattice(d, dims, precision, seed=2)
    L.set_populations(f0)
    L.set_correlation(0)
    L.set_correlation(5, ks, 2)
    a = L.fourier_amplitudes()
    L.close()
    ref = oracle.population_amplitudes(f0.astype(np.float64), ks)
    A = _scale(f0)
    err = np.abs(a - ref) / A[None, :]
    print(f"[corr] amplitudes D{d} {dims} fp{8 * precision}: max {err.max():.2e}", flush=True)
    assert err.max() < 1e-13


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("d,dims", CASES)
def test_correlators_match_oracle(d, dims, precision):
    dt = np.float32 if precision == 4 else np.float64
    f0 = poisson_state(d, dims, 10.0, seed=6).astype(dt)
    ks = np.array(KS[d])
    steps, every, nlag, t0 = 13, 3, 4, 2
    L = gpu_lattice(d, dims, precision, omega=1.3, seed=9)
    L.set_populations(f0, step=t0)
    L.set_correlation(every, ks, nlag)
    L.step(steps)
    sij, ct, n = L.correlation()
    L.close()
    res = oracle.correlate(f0.astype(np.float64), oracle.Params(d=d, omega_j=1.3, seed=9), steps, ks, every,
                           nlag, t0=t0)
    assert n == res["nsamples"] == len([t for t in range(t0, t0 + steps) if t % every == 0])
    A = _scale(f0)
    scale = n * np.outer(A, A)[None]
    es = np.abs(sij - res["sij"]) / scale
    ec = np.abs(ct - res["ct"]) / (n * A.sum() ** 2)
    print(f"[corr] D{d} {dims} fp{8 * precision}: S_ij {es.max():.2e}  C {ec.max():.2e}", flush=True)
    assert es.max() < TOL[precision]
    assert ec.max() < TOL[precision]


def test_full_size_amplitudes():
    # the 4096^2 FP32 lattice of the benchmark, seeded Poisson state
    dims = (4096, 4096)
    f0 = poisson_state(2, dims, 10.0, seed=12).astype(np.float32)
    ks = np.array([[0, 0], [1, 0], [0, 1], [3, 5], [2048, 2048], [-7, 100]])
    L = gpu_lattice(2, dims, 4, seed=1)
    L.set_populations(f0)
    L.set_correlation(10, ks, 1)
    a = L.fourier_amplitudes()
    L.close()
    ref = oracle.population_amplitudes(f0.astype(np.float64), ks)
    err = np.abs(a - ref) / _scale(f0)[None, :]
    print(f"[corr] amplitudes 4096^2 fp32: max {err.max():.2e}", flush=True)
    assert err.max() < 1e-13


def test_edge_cases_and_errors():
    f0 = poisson_state(1, (64,), 5.0, seed=1)
    L = gpu_lattice(1, (64,), 8)
    L.set_populations(f0)
    with pytest.raises(flb.FlbError) as e:
        L.correlation()
    assert e.value.code == flb.FLB_ESTATE
    for bad in (dict(kvecs=np.zeros((0, 1)), nlag=1), dict(kvecs=[[1]], nlag=0),
                dict(kvecs=[[1]], nlag=70000), dict(kvecs=np.zeros((1025, 1)), nlag=1),
                dict(kvecs=np.zeros((1000, 1)), nlag=2000)):
        with pytest.raises(flb.FlbError) as e:
            L.set_correlation(1, **bad)
        assert e.value.code == flb.FLB_EINVAL
    # more lags than samples: the missing lags stay zero; k = 0 is the mass squared
    L.set_correlation(1, [[0], [5]], 8)
    L.step(3)
    sij, ct, n = L.correlation()
    assert n == 3
    assert np.all(ct[:, 3:] == 0) and np.all(ct[:, :3] != 0)
    M = f0.sum()
    assert abs(ct[0, 0] - 3 * M * M) < 1e-12 * M * M
    assert abs(sij[0].sum() - 3 * M * M) < 1e-12 * M * M
    # stopping keeps the sums; sampling period longer than the run: no samples
    L.set_correlation(0)
    L.step(4)
    assert L.correlation()[2] == 3
    L.set_correlation(100, [[1]], 1)
    L.step(50)                         # steps 7..56: no multiple of 100
    sij, ct, n = L.correlation()
    assert n == 0 and np.all(sij == 0) and np.all(ct == 0)
    L.close()


def test_sampling_kinds_do_not_interfere():
    # correlators, lattice sums and S(k) sampled together equal each alone,
    # and the trajectory is unchanged by sampling
    d, dims = 2, (96, 40)
    f0 = poisson_state(d, dims, 8.0, seed=2)
    ks = [[1, 0], [2, 3]]

    def run(corr, mom, sk):
        L = gpu_lattice(d, dims, 8, seed=4)
        L.set_populations(f0)
        if corr:
            L.set_correlation(2, ks, 3)
        if mom:
            L.set_moment_sampling(3)
        if sk:
            L.set_sampling(2, ks)
        L.step(11)
        out = {"f": L.get_populations()}
        if corr:
            out["corr"] = L.correlation()
        if mom:
            out["mom"] = L.sampled_moments()[0]["sum_ff"]
        if sk:
            out["sk"] = L.structure_factor(mode="read")[:2]
        L.close()
        return out

    both = run(True, True, True)
    plain = run(False, False, False)
    assert np.array_equal(both["f"], plain["f"])
    c = run(True, False, False)["corr"]
    assert np.array_equal(both["corr"][0], c[0]) and np.array_equal(both["corr"][1], c[1])
    assert np.array_equal(both["mom"], run(False, True, False)["mom"])
    assert np.array_equal(both["sk"], run(False, False, True)["sk"])


def _batch_means(x, nb):
    x = np.asarray(x)
    m = len(x) // nb
    return x[: nb * m].reshape(nb, m, *x.shape[1:]).mean(axis=1)


def test_fourier_test_flat_fig2():
    # D2Q5, L = 10, rho = 120, unit rates, the paper's flat noise law, local
    # noise.  S_ij^diff(k) = S_ij(k) - S_ij^th(k) shows no structure: every
    # normalised entry is consistent with zero within its batch-means error.
    d, side, rho = 2, 10, 120.0
    lat = oracle.make_lattice(d)
    N = side * side
    ks = np.array([[kx, ky] for ky in range(side) for kx in range(side)])
    nb, per = 20, 10000
    f0 = inputs.outer(lat.w, np.full((side, side), rho))
    L = gpu_lattice(d, (side, side), 8, seed=77, law="uniform")
    L.set_populations(f0)
    L.step(200)
    batches = []
    prev = None
    L.set_correlation(1, ks, 1)
    for _ in range(nb):
        L.step(per)
        sij, _, n = L.correlation()
        cur = sij.copy()
        batches.append((cur - (prev if prev is not None else 0)) / per)
        prev = cur
    L.close()
    B = np.array(batches)                                   # (nb, nk, Q, Q)
    feq = rho * lat.w
    th = np.zeros((len(ks), 5, 5))
    for j, k in enumerate(ks):
        if k[0] == 0 and k[1] == 0:
            th[j] = N * N * np.outer(feq, feq)
        else:
            th[j] = N * np.diag(feq)
    diff = B.real - th[None]
    norm = N * np.sqrt(np.outer(feq, feq))[None, None]
    z = diff.mean(axis=0) / (diff.std(axis=0, ddof=1) / np.sqrt(nb))
    nonzero = np.array([not (k[0] == 0 and k[1] == 0) for k in ks])
    zz = z[nonzero]
    print(f"[fig2] mean |S_diff|/(N f_eq) {np.abs(diff.mean(axis=0)[nonzero] / norm[0]).mean():.2e}, "
          f"max |z| {np.abs(zz).max():.2f}, mean z^2 {np.mean(zz ** 2):.2f}", flush=True)
    assert np.mean(zz ** 2) < 1.6
    assert np.abs(zz).max() < 6.0
    # k = 0 is deterministic: total mass squared
    k0 = np.flatnonzero(~nonzero)[0]
    assert abs(B[:, k0].real.sum(axis=(1, 2)).mean() / (N * rho) ** 2 - 1) < 1e-12
    # overall level: diagonal S_ii / (N f_i^eq) = 1 to the statistical error
    diag = np.array([np.real(np.diag(B[:, j].mean(axis=0))) / (N * feq) for j in np.flatnonzero(nonzero)])
    assert np.abs(diag.mean(axis=0) - 1).max() < 0.01


def test_time_correlator_fig7():
    # <rho(k, 0) rho(-k, t)> / <|rho(k)|^2> = lambda(k)^t at unit rates
    # (the exact discrete form of eq. TimeCorrEqn's exponential)
    d, dims, rho = 2, (32, 32), 50.0
    lat = oracle.make_lattice(d)
    ks = np.array([[1, 0], [0, 2], [2, 2], [4, 1], [8, 0]])
    nlag = 24
    f0 = inputs.outer(lat.w, np.full((32, 32), rho))
    L = gpu_lattice(d, dims, 8, seed=5)
    L.set_populations(f0)
    L.step(300)
    nb, per = 16, 12000
    prev_ct, prev_n = None, 0
    ratios = []
    L.set_correlation(1, ks, nlag)
    for _ in range(nb):
        L.step(per)
        _, ct, n = L.correlation()
        cur = ct.copy()
        seg = cur - (prev_ct if prev_ct is not None else 0)
        ratios.append(seg.real / seg.real[:, :1])
        prev_ct, prev_n = cur, n
    L.close()
    R = np.array(ratios)                                   # (nb, nk, nlag)
    mean, err = R.mean(axis=0), R.std(axis=0, ddof=1) / np.sqrt(nb)
    worst = 0.0
    for j, k in enumerate(ks):
        lam = cf.ftcs_factor(lat.theta, k, dims)
        expect = lam ** np.arange(nlag)
        z = (mean[j] - expect)[1:] / np.maximum(err[j][1:], 1e-4)
        worst = max(worst, np.abs(z).max())
        print(f"[fig7] k={tuple(k)} lambda={lam:.5f}: C(10)/C(0) {mean[j, 10]:.4f} vs {expect[10]:.4f}",
              flush=True)
        assert np.abs(mean[j] - expect).max() < 0.02
    assert worst < 6.0
