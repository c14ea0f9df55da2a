"""Batched ensembles: each member's state after a batched run must be
bit-identical to the same lattice stepped alone (and therefore within the
oracle tolerance, checked for a few members); graph replay must equal eager
launches; members can be admitted and retired between calls."""

import numpy as np
import pytest

import oracle
from paper_1606_07801_amd import flb, inputs
from tests.gpu_common import RTOL, report, scaled_error

pytestmark = pytest.mark.gpu


def _member(spec, precision):
    d, dims, omega, rho, seed = spec
    lat = oracle.make_lattice(d)
    f0 = inputs.poisson_counts(dims, rho * lat.w, seed=seed).astype(np.float32 if precision == 4 else np.float64)
    return f0, dict(omega=omega, seed=seed, noise="local")


def _specs():
    gen = np.random.default_rng(5)
    out = []
    # small D1Q3 (LDS-resident), a large D1Q3 (global), D2Q5 and D3Q7 of uneven sizes
    for L in (64, 100, 1000, 4096, 3333):
        out.append((1, (L,), float(gen.uniform(0.5, 1.9)), float(gen.uniform(0.1, 50)), int(gen.integers(1, 1 << 40))))
    out.append((1, (20000,), 1.3, 7.0, 17))
    for dims in ((128, 130), (300, 17), (257, 64)):
        out.append((2, dims, float(gen.uniform(0.5, 1.9)), float(gen.uniform(0.1, 50)), int(gen.integers(1, 1 << 40))))
    out.append((3, (40, 33, 17), 1.1, 5.0, 99))
    return out


def _alone(specs, precision, nsteps, t0):
    res = []
    for spec in specs:
        f0, kw = _member(spec, precision)
        L = flb.Lattice(spec[0], spec[1], precision=precision, **kw)
        L.set_populations(f0, step=t0)
        L.step(nsteps)
        res.append(L.get_populations())
        L.close()
    return res


@pytest.mark.parametrize("precision", [4, 8])
@pytest.mark.parametrize("use_graph,tiling,depth,chunk,width", [
    (True, 0, 2, 16, 256), (False, 0, 2, 16, 256), (True, 1, 1, 16, 256), (True, 0, 1, 16, 256),
    (True, 0, 2, 7, 256), (True, 0, 2, 16, 128), (True, 0, 2, 7, 64)])
def test_batch_bit_identical_to_alone(precision, use_graph, tiling, depth, chunk, width):
    # depth 2: D2Q5 members in two-step passes (tiles of `width` columns); odd
    # chunks and remainders end with a single step
    specs = _specs()
    nsteps, t0 = 37, 5           # chunks of 16 (or 7) + a remainder
    ref = _alone(specs, precision, nsteps, t0)
    B = flb.Batch(chunk=chunk, use_graph=use_graph, tiling=tiling, depth=depth, width=width)
    lats = []
    for spec in specs:
        f0, kw = _member(spec, precision)
        L = flb.Lattice(spec[0], spec[1], precision=precision, **kw)
        L.set_populations(f0, step=t0)
        B.admit(L)
        lats.append(L)
    assert len(B) == len(specs)
    B.step(nsteps)
    B.sync()
    for L, r, spec in zip(lats, ref, specs):
        B.retire(L)
        assert L.t == t0 + nsteps
        g = L.get_populations()
        assert np.array_equal(g.view(np.uint8), r.view(np.uint8)), spec
        L.close()
    B.close()


@pytest.mark.parametrize("precision", [4, 8])
@pytest.mark.parametrize("plans", [("local", "gauss"), ("global", "gauss"), ("local", "uniform"), ("off", "gauss")])
def test_batch_noise_plans(precision, plans):
    # D2Q5 members at depth 2: an all local-Gaussian batch runs the instances
    # with that noise plan fixed at compile time; one member of another plan
    # switches the batch to reading it from the parameters
    noise, law = plans
    members = [((128, 130), 1.3, 8.0, 3, "local", "gauss"), ((300, 17), 0.9, 20.0, 4, noise, law),
               ((257, 64), 1.7, 2.0, 5, "local", "gauss")]
    nsteps, t0 = 21, 3
    dt = np.float32 if precision == 4 else np.float64
    w = oracle.make_lattice(2).w

    def make(m):
        dims, omega, rho, seed, nz, lw = m
        L = flb.Lattice(2, dims, precision=precision, omega=omega, seed=seed, noise=nz, law=lw)
        L.set_populations(inputs.poisson_counts(dims, rho * w, seed=seed).astype(dt), step=t0)
        return L

    ref = []
    for m in members:
        L = make(m)
        L.step(nsteps)
        ref.append(L.get_populations())
        L.close()
    B = flb.Batch(chunk=8, depth=2)
    lats = [make(m) for m in members]
    for L in lats:
        B.admit(L)
    B.step(nsteps)
    B.sync()
    for L, r, m in zip(lats, ref, members):
        B.retire(L)
        assert np.array_equal(L.get_populations().view(np.uint8), r.view(np.uint8)), m
        L.close()
    B.close()


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("width", [256, 64])
def test_batch_members_match_oracle(precision, width):
    # every kind of member against the oracle: D1Q3 in LDS, D2Q5 in two-step
    # passes over tiles of `width` columns (an odd step count ends with a
    # single flat step), D3Q7 in flat items; densities >= 5, away from the
    # non-Lipschitz amplitude at rho = 0
    specs = [(1, (64,), 1.3, 9.0, 11), (1, (1000,), 0.7, 6.0, 12), (1, (4096,), 1.8, 30.0, 13),
             (2, (128, 130), 1.1, 8.0, 21), (2, (300, 17), 0.6, 20.0, 22), (2, (257, 64), 1.7, 12.0, 23),
             (3, (40, 33, 17), 1.1, 5.0, 99)]
    B = flb.Batch(chunk=8, depth=2, width=width)
    lats, f0s = [], []
    for spec in specs:
        f0, kw = _member(spec, precision)
        L = flb.Lattice(spec[0], spec[1], precision=precision, **kw)
        L.set_populations(f0)
        B.admit(L)
        lats.append(L)
        f0s.append(f0)
    B.step(21)
    for L, f0, spec in zip(lats, f0s, specs):
        B.retire(L)
        g = L.get_populations()
        p = oracle.Params(d=spec[0], omega_j=spec[2], seed=spec[4])
        fo = oracle.run(f0.astype(np.float64), p, 21)
        err = scaled_error(g, fo, spec[3], p.lattice().w)
        assert report(f"batch member fp{8 * precision} width {width} D{spec[0]} {spec[1]}", err) <= RTOL[precision]
        L.close()
    B.close()


def test_admit_refuses_sampling_lattices():
    # a batch step takes no statistics: a lattice that samples S(k), lattice
    # sums or correlators while stepping is refused rather than silently
    # left unsampled
    B = flb.Batch()
    for setup in (lambda L: L.set_sampling(5, [(1, 0)]), lambda L: L.set_moment_sampling(3),
                  lambda L: L.set_correlation(4, [(1, 0)], nlag=2)):
        L = flb.Lattice(2, (32, 16), precision=4)
        L.set_populations(np.ones((5, 16, 32), dtype=np.float32))
        setup(L)
        with pytest.raises(flb.FlbError) as e:
            B.admit(L)
        assert e.value.code == flb.FLB_ESTATE
        L.close()
    assert len(B) == 0
    B.close()


def test_admit_retire_between_calls():
    # a member that joins late or leaves early ends where it would alone
    specs = _specs()[:6] + _specs()[6:8]
    ref_a = _alone(specs, 4, 30, 0)
    B = flb.Batch(chunk=4)
    lats = []
    for i, spec in enumerate(specs):
        f0, kw = _member(spec, 4)
        L = flb.Lattice(spec[0], spec[1], precision=4, **kw)
        L.set_populations(f0)
        lats.append(L)
    first, late = lats[: len(lats) // 2], lats[len(lats) // 2:]
    for L in first:
        B.admit(L)
    B.step(10)
    for L in late:       # late members step 10 alone first
        L.step(10)
        L.sync()
        B.admit(L)
    B.step(13)
    B.retire(first[0])   # one member leaves, finishes alone
    first[0].step(7)
    B.step(7)
    for L in lats:
        if L is not first[0]:
            B.retire(L)
    for L, r in zip(lats, ref_a):
        assert L.t == 30
        assert np.array_equal(L.get_populations(), r)
        L.close()
    B.close()


def test_batch_errors():
    for bad in (dict(width=96), dict(width=512), dict(depth=3)):
        with pytest.raises(flb.FlbError) as e:
            flb.Batch(**bad)
        assert e.value.code == flb.FLB_EINVAL
    B = flb.Batch()
    a = flb.Lattice(1, (64,), precision=4)
    b = flb.Lattice(1, (64,), precision=8)
    a.set_populations(np.ones((3, 64), dtype=np.float32))
    B.admit(a)
    with pytest.raises(flb.FlbError) as e:
        B.admit(b)                    # mixed precision
    assert e.value.code == flb.FLB_EINVAL
    with pytest.raises(flb.FlbError) as e:
        a.step(1)                     # a member is stepped by its batch only
    assert e.value.code == flb.FLB_ESTATE
    with pytest.raises(flb.FlbError):
        B.admit(a)                    # already a member
    with pytest.raises(flb.FlbError):
        B.retire(b)                   # not a member
    B.retire(a)
    a.step(1)
    a.close()
    b.close()
    B.close()


def test_lds_path_equals_global_path():
    # the same small D1Q3 lattices with the LDS path disabled
    specs = [s for s in _specs() if s[0] == 1 and s[1][0] <= 4096]
    outs = []
    for lds in (0, -1):
        B = flb.Batch(chunk=16, lds_max_bytes=lds)
        lats = []
        for spec in specs:
            f0, kw = _member(spec, 4)
            L = flb.Lattice(1, spec[1], precision=4, **kw)
            L.set_populations(f0)
            B.admit(L)
            lats.append(L)
        B.step(40)
        res = []
        for L in lats:
            B.retire(L)
            res.append(L.get_populations())
            L.close()
        B.close()
        outs.append(res)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
