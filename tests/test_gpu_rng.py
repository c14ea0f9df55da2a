"""The device noise stream against the oracle (bit-exact Philox words) and
the oracle's Philox against an independent library implementation."""

import ctypes
import os

import numpy as np
import pytest

import oracle
from oracle import philox
from paper_1606_07801_amd import flb

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("seed,step,site0", [(0, 0, 0), (12345, 7, 1000), ((1 << 63) + 99, (1 << 32) - 1, 0),
                                             (42, 3, (1 << 32) - 3000), (7, 123456789, (1 << 40) + 5)])
def test_words_bit_exact(d, seed, step, site0):
    n = 6000
    words, _ = flb.noise_sample(d, seed, step, site0, n, precision=8)
    sites = np.arange(site0, site0 + n, dtype=np.uint64)
    nblk = 2 if d == 3 else 1
    for b in range(nblk):
        r = philox.philox4x32_10(sites & np.uint64(0xFFFFFFFF), sites >> np.uint64(32),
                                 step & 0xFFFFFFFF, b, seed & 0xFFFFFFFF, seed >> 32)
        for k in range(4):
            assert np.array_equal(words[4 * b + k].astype(np.uint64), r[k])


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("law", ["gauss", "uniform"])
def test_variates_match_oracle(d, law):
    n = 20000
    lat = oracle.make_lattice(d)
    ref = oracle.noise_draws(lat, 99, 5, np.arange(n, dtype=np.uint64) + 10, law=law)
    for prec, tol in ((8, 1e-14), (4, 1e-6)):
        _, v = flb.noise_sample(d, 99, 5, 10, n, precision=prec, law=law)
        # uniform law: the device returns 2u - 1
        r = ref if law == "gauss" else 2 * ref - 1
        err = np.abs(v.astype(np.float64) - r) / np.maximum(1.0, np.abs(r))
        print(f"[rng] D{d} {law} fp{8 * prec}: max rel err {err.max():.3e}", flush=True)
        assert err.max() <= tol


def _rocrand():
    for path in ("/opt/rocm/lib/librocrand.so", "/opt/rocm/lib/librocrand.so.1"):
        if os.path.exists(path):
            return ctypes.CDLL(path)
    return None


def test_oracle_philox_matches_rocrand_host_generator():
    # Independent implementation: rocRAND's Philox4x32-10 host generator, used
    # as a black box.  Its stream for a seed s and offset 0 is taken as the
    # words of counters (j, 0, 0, 0), j = 0, 1, ..., under key (s lo, s hi).
    lib = _rocrand()
    if lib is None:
        pytest.skip("rocRAND not installed")
    gen = ctypes.c_void_p()
    st = lib.rocrand_create_generator_host_blocking(ctypes.byref(gen), 404)  # PHILOX4_32_10
    if st != 0:
        pytest.skip(f"rocRAND host generator unavailable (status {st})")
    try:
        for seed in (0, 1, 0x0123456789ABCDEF):
            assert lib.rocrand_set_seed(gen, ctypes.c_ulonglong(seed)) == 0
            assert lib.rocrand_set_offset(gen, ctypes.c_ulonglong(0)) == 0
            n = 4096
            out = np.zeros(4 * n, dtype=np.uint32)
            st = lib.rocrand_generate(gen, out.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(out.size))
            assert st == 0, st
            j = np.arange(n, dtype=np.uint64)
            r = philox.philox4x32_10(j, 0, 0, 0, seed & 0xFFFFFFFF, seed >> 32)
            mine = np.stack([x.astype(np.uint32) for x in r], axis=1).ravel()
            print(f"[rocrand] seed {seed:#x}: first words {out[:4]} oracle {mine[:4]}", flush=True)
            assert np.array_equal(out, mine)
    finally:
        lib.rocrand_destroy_generator(gen)


def test_gauss_map_exhaustive():
    # every uniform u0 and every uniform u1 (2^23 values each; the low nine
    # bits of a word do not enter), paired by a seeded permutation, against the
    # oracle's Box-Muller in FP64 and, on a sample, against 40-digit values
    gen = np.random.default_rng(17)
    j = np.arange(1 << 23, dtype=np.uint32)
    r0 = (j << np.uint32(9)) | gen.integers(0, 512, j.size, dtype=np.uint32)
    r1 = (gen.permutation(j) << np.uint32(9)) | gen.integers(0, 512, j.size, dtype=np.uint32)
    u0, u1 = philox.words_to_uniform(r0), philox.words_to_uniform(r1)
    c_ref, s_ref = philox.box_muller(u0, u1)
    R = np.sqrt(-2.0 * np.log(u0))
    scale = np.maximum(1.0, R)
    for prec, tol in ((8, 2e-15), (4, 1e-6)):
        z0, z1 = flb.gauss_map(r0, r1, precision=prec)
        e = max((np.abs(z0.astype(np.float64) - c_ref) / scale).max(),
                (np.abs(z1.astype(np.float64) - s_ref) / scale).max())
        print(f"[rng] gauss map fp{8 * prec}, all 2^23 u0 and u1: max |err| / max(1, R) = {e:.3e}", flush=True)
        assert e <= tol
        if prec == 8:
            try:
                import mpmath
            except ImportError:
                continue
            mpmath.mp.dps = 40
            pick = np.concatenate([gen.integers(0, j.size, 1500), np.argsort(u0)[:5], np.argsort(u0)[-5:],
                                   np.argsort(u1)[:5], np.argsort(u1)[-5:]])
            worst = 0.0
            for t in pick:
                a = mpmath.mpf(int(((int(r0[t]) >> 9) << 1) | 1)) / 2 ** 24
                b = mpmath.mpf(int(((int(r1[t]) >> 9) << 1) | 1)) / 2 ** 24
                rr = mpmath.sqrt(-2 * mpmath.log(a))
                worst = max(worst, abs(float(rr * mpmath.cos(2 * mpmath.pi * b)) - z0[t]) / max(1.0, float(rr)),
                            abs(float(rr * mpmath.sin(2 * mpmath.pi * b)) - z1[t]) / max(1.0, float(rr)))
            print(f"[rng] gauss map fp64 vs 40-digit values: {worst:.3e}", flush=True)
            assert worst <= 1e-15
