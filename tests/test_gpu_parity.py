"""GPU parity: the HIP step through the C ABI against the FP64 oracle on the
same seeded inputs, element by element (tolerance semantics in gpu_common)."""

import numpy as np
import pytest

import oracle
from paper_1606_07801_amd import flb, inputs
from tests.gpu_common import RTOL, poisson_state, report, run_both, scaled_error, gpu_lattice

pytestmark = pytest.mark.gpu

# ragged sizes spanning several 256-wide tiles and partial row groups
SIZES = {1: (1000,), 2: (300, 70), 3: (40, 33, 17)}


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("noise,law", [("local", "gauss"), ("global", "gauss"),
                                       ("local", "uniform"), ("off", "gauss")])
def test_multistep_parity(d, precision, noise, law):
    dims = SIZES[d]
    f0 = poisson_state(d, dims, 10.0, seed=d)
    g, fo, w, _ = run_both(d, dims, precision, 25, f0, t0=3, omega=1.3, seed=77, noise=noise, law=law)
    err = scaled_error(g, fo, 10.0, w)
    assert report(f"D{d} fp{8 * precision} {noise}/{law} 25 steps", err) <= RTOL[precision]


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_mrt_classes_parity(d, precision):
    dims = SIZES[d]
    f0 = poisson_state(d, dims, 20.0, seed=5)
    g, fo, w, _ = run_both(d, dims, precision, 20, f0, omega=0.6, omega_n=1.5, omega_s=1.9, seed=3)
    assert report(f"D{d} fp{8 * precision} MRT", scaled_error(g, fo, 20.0, w)) <= RTOL[precision]


@pytest.mark.parametrize("d", [1, 2, 3])
def test_theta_parameter_parity(d):
    th = {1: 0.45, 2: 0.2, 3: 0.3}[d]
    dims = SIZES[d]
    lat = oracle.make_lattice(d, th)
    f0 = inputs.poisson_counts(dims, 10.0 * lat.w, seed=1)
    g, fo, w, _ = run_both(d, dims, 8, 15, f0, omega=1.1, seed=9, theta=th)
    assert report(f"D{d} theta={th}", scaled_error(g, fo, 10.0, w)) <= RTOL[8]


@pytest.mark.parametrize("d", [1, 2, 3])
def test_seed_high_word_and_step_keying(d):
    dims = SIZES[d]
    f0 = poisson_state(d, dims, 10.0, seed=2)
    seed = (0xDEADBEEF << 32) | 0x12345678
    g, fo, w, _ = run_both(d, dims, 8, 3, f0, t0=(1 << 32) - 2, omega=1.0, seed=seed)
    assert report(f"D{d} step wrap, 64-bit seed", scaled_error(g, fo, 10.0, w)) <= RTOL[8]


@pytest.mark.parametrize("precision", [8, 4])
def test_low_density_parity(precision):
    # rho = 0.1: ~half the sites pass through rho <= 0, where sqrt(max(rho, 0))
    # turns rounding differences of rho into O(sqrt(eps)) differences of the
    # noise amplitude.  Global noise and noise off stay within the tolerance
    # everywhere; local noise is compared per population for one step from
    # identical inputs, and over many steps statistically (test_gpu_stats).
    d, dims = 2, SIZES[2]
    f0 = poisson_state(d, dims, 0.1, seed=11)
    for noise in ("global", "off"):
        g, fo, w, _ = run_both(d, dims, precision, 20, f0, omega=1.0, seed=4, noise=noise)
        assert report(f"rho=0.1 {noise} fp{8 * precision}", scaled_error(g, fo, 0.1, w)) <= RTOL[precision]
    g, fo, w, _ = run_both(d, dims, precision, 1, f0, omega=1.0, seed=4, noise="local")
    assert report(f"rho=0.1 local 1 step fp{8 * precision}", scaled_error(g, fo, 0.1, w)) <= RTOL[precision]
    g, fo, w, _ = run_both(d, dims, precision, 20, f0, omega=1.0, seed=4, noise="local")
    err = scaled_error(g, fo, 0.1, w)
    frac = float(np.mean(err > RTOL[precision]))
    mx = report(f"rho=0.1 local 20 steps fp{8 * precision} (fraction above tol {frac:.2e})", err)
    if precision == 8:
        # a few sites whose density passed within rounding of zero: the
        # amplitude sqrt(max(rho, 0)) turns a 1e-17 difference of rho into
        # ~1e-9 of the noise (measured: fraction 5e-4, max 9e-12)
        assert frac <= 2e-3 and mx <= 1e-10
    else:
        assert frac < 0.05


@pytest.mark.parametrize("law", ["uniform", "gauss"])
def test_low_density_fp64_many_steps(law):
    # rho = 0.1, local noise, FP64, 20 steps: the flat law's variates are
    # exact in both implementations (2u - 1 of an exact u), the Gaussian
    # map's carry the rounding of the device's and numpy's logarithm and
    # sine; either way the only amplification is the non-Lipschitz amplitude
    # at rho = 0, which stays at a few sites
    d, dims = 2, SIZES[2]
    f0 = poisson_state(d, dims, 0.1, seed=11)
    g, fo, w, _ = run_both(d, dims, 8, 20, f0, omega=1.0, seed=4, noise="local", law=law)
    err = scaled_error(g, fo, 0.1, w)
    frac = float(np.mean(err > RTOL[8]))
    mx = report(f"rho=0.1 local/{law} 20 steps fp64 (fraction above 1e-12: {frac:.2e})", err)
    assert frac <= 2e-3 and mx <= 1e-10


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_kernel_variants_bit_identical(d, precision):
    dims = SIZES[d]
    f0 = poisson_state(d, dims, 10.0, seed=3).astype(np.float32 if precision == 4 else np.float64)
    outs = []
    for kern, tx, ry, nt, pp in [("plain", 0, 0, 0, 0), ("rows", 256, 4, 0, 0), ("rows", 64, 1, 1, 0),
                                 ("rows", 1024, 16, 0, 0), ("rows", 128, 8, 1, 0), ("rows", 512, 2, 0, 0),
                                 ("rows", 256, 16, 1, 0), ("rows", 256, 4, 1, 1), ("rows", 128, 16, 0, 1),
                                 ("flat", 0, 1, 0, 0), ("flat", 0, 2, 1, 0), ("flat", 0, 8, 1, 0)]:
        L = gpu_lattice(d, dims, precision, omega=1.2, seed=5, kernel=kern, tile_x=tx, tile_rows=ry, nt_store=nt,
                        pipeline=pp)
        L.set_populations(f0)
        L.step(12)
        outs.append(L.get_populations())
        L.close()
    for o in outs[1:]:
        assert np.array_equal(o.view(np.uint8), outs[0].view(np.uint8))


def test_split_runs_equal_one_run():
    # checkpoint / resume: n + m steps in one go equal n steps, a state
    # round-trip through host memory into a new handle, then m steps
    d, dims = 2, SIZES[2]
    f0 = poisson_state(d, dims, 10.0, seed=8)
    A = gpu_lattice(d, dims, 4, omega=1.4, seed=21)
    A.set_populations(f0)
    A.step(17)
    a = A.get_populations()
    B = gpu_lattice(d, dims, 4, omega=1.4, seed=21)
    B.set_populations(f0)
    B.step(9)
    mid = B.get_populations()
    t = B.t
    B.close()
    C = gpu_lattice(d, dims, 4, omega=1.4, seed=21)
    C.set_populations(mid, step=t)
    C.step(8)
    assert np.array_equal(C.get_populations(), a)
    A.close()
    C.close()


def test_set_get_roundtrip_and_zero_steps():
    for d in (1, 2, 3):
        dims = SIZES[d]
        f0 = np.random.default_rng(d).normal(size=(2 * d + 1,) + tuple(reversed(dims)))
        L = gpu_lattice(d, dims, 8)
        L.set_populations(f0)
        L.step(0)
        assert np.array_equal(L.get_populations(), f0)
        L.close()


def test_degenerate_sizes():
    # sizes 1 and 2 along an axis: the periodic neighbours coincide
    for d, dims in [(1, (1,)), (1, (2,)), (2, (1, 5)), (2, (7, 1)), (2, (2, 2)), (3, (1, 1, 1)),
                    (3, (3, 1, 2))]:
        f0 = poisson_state(d, dims, 10.0, seed=1)
        g, fo, w, _ = run_both(d, dims, 8, 6, f0, omega=1.5, seed=2)
        assert report(f"D{d} {dims}", scaled_error(g, fo, 10.0, w)) <= RTOL[8]


def test_errors_from_device_calls():
    L = gpu_lattice(2, (16, 8), 4)
    with pytest.raises(flb.FlbError):
        L.step(-1)
    with pytest.raises(ValueError):
        L.set_populations(np.zeros((5, 8, 15), dtype=np.float32))
    with pytest.raises(flb.FlbError) as e:
        L.structure_factor(None, mode="read")
    assert e.value.code == flb.FLB_ESTATE
    L.close()


@pytest.mark.parametrize("kernel,dims", [("two", (300, 70)), ("auto", (60, 40)), ("flat", (1000,))])
def test_check_mode_reports_nonfinite(kernel, dims):
    # a NaN set through flb_set_populations: with checks every step the next
    # step stops with FLB_ENONFINITE at step 1; every 4 steps, at step 4
    d = len(dims)
    f0 = poisson_state(d, dims, 10.0, seed=3).astype(np.float32)
    for every, stop in ((1, 1), (4, 4)):
        bad = f0.copy()
        bad.reshape(-1)[123] = np.nan
        L = gpu_lattice(d, dims, 4, kernel=kernel)
        L.set_populations(bad)
        L.set_check(every)
        with pytest.raises(flb.FlbError) as e:
            L.step(10)
        assert e.value.code == flb.FLB_ENONFINITE and L.t == stop, (every, L.t)
        L.close()
    # a finite state passes the checks, with results equal to unchecked steps
    A = gpu_lattice(d, dims, 4, kernel=kernel)
    B = gpu_lattice(d, dims, 4, kernel=kernel)
    for L in (A, B):
        L.set_populations(f0)
    A.set_check(3)
    A.step(10)
    B.step(10)
    assert A.t == 10 and np.array_equal(A.get_populations(), B.get_populations())
    A.close()
    B.close()
