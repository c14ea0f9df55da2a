"""Pins of the oracle's Philox4x32-10 and its uniform / Gaussian mappings.

The round structure is cross-checked against an independent library build of
Philox4x32-10 in tests/test_gpu_rng.py (needs the GPU runtime).  Here: the
constants that have a definition, and distribution tests that a wrong
constant, shift or word order would fail."""

import decimal

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import philox


def _frac_bits(x):
    decimal.getcontext().prec = 60
    return int((x - int(x)) * (decimal.Decimal(2) ** 32))


def test_weyl_constants_from_definition():
    decimal.getcontext().prec = 60
    phi = (1 + decimal.Decimal(5).sqrt()) / 2
    assert _frac_bits(phi) == int(philox.PHILOX_W0)
    assert _frac_bits(decimal.Decimal(3).sqrt()) == int(philox.PHILOX_W1)


def test_multipliers_are_odd_32bit():
    for mlt in (philox.PHILOX_M0, philox.PHILOX_M1):
        assert int(mlt) % 2 == 1 and int(mlt) < 2 ** 32


def _words(n, seed=12345, step=7, block=0):
    site = np.arange(n, dtype=np.uint64)
    return philox.philox4x32_10(site & np.uint64(0xFFFFFFFF), site >> np.uint64(32),
                                step, block, seed & 0xFFFFFFFF, seed >> 32)


def test_word_bits_balanced():
    r = np.concatenate(_words(1 << 16))
    bits = np.unpackbits(r.astype(">u4").view(np.uint8)).reshape(-1, 32)
    p = bits.mean(axis=0)
    # 262144 samples per bit: std of the mean is ~1e-3
    assert np.abs(p - 0.5).max() < 6e-3


def test_bytes_uniform_chi2():
    r = np.concatenate(_words(1 << 15)).astype(np.uint32)
    for shift in (0, 8, 16, 24):
        h = np.bincount((r >> shift) & 0xFF, minlength=256)
        chi2, pval = stats.chisquare(h)
        assert pval > 1e-4


def test_avalanche_on_counter_and_key():
    n = 4096
    base = np.array(_words(n, seed=99)).astype(np.uint32)
    site = np.arange(n, dtype=np.uint64)
    for bit in (0, 13, 31):
        flipped = philox.philox4x32_10(site ^ np.uint64(1 << bit), 0, 7, 0, 99, 0)
        diff = np.array(flipped).astype(np.uint32) ^ base
        frac = np.unpackbits(diff.view(np.uint8)).mean()
        assert abs(frac - 0.5) < 0.01
    for bit in (0, 31):
        flipped = philox.philox4x32_10(site, 0, 7, 0, 99 ^ (1 << bit), 0)
        diff = np.array(flipped).astype(np.uint32) ^ base
        assert abs(np.unpackbits(diff.view(np.uint8)).mean() - 0.5) < 0.01


def test_words_differ_across_step_block_and_key():
    a = np.array(_words(1024, step=0, block=0))
    for other in (_words(1024, step=1, block=0), _words(1024, step=0, block=1),
                  _words(1024, seed=12346, step=0, block=0)):
        assert np.mean(a == np.array(other)) < 1e-3


def test_uniform_mapping_exact_and_open():
    r = np.array([0, 1, 511, 512, 0xFFFFFFFF, 0x80000000], dtype=np.uint64)
    u = philox.words_to_uniform(r)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24 and u[2] == 2.0 ** -24
    assert u[3] == 3 * 2.0 ** -24
    assert u[4] == 1 - 2.0 ** -24
    assert u[5] == 0.5 + 2.0 ** -24
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    assert np.all((u > 0) & (u < 1))


def test_box_muller_normal_law():
    lat = oracle.make_lattice(2)
    z = oracle.noise_draws(lat, seed=5, t=3, sites=np.arange(200_000))
    assert z.shape == (4, 200_000)
    for row in z:
        assert abs(row.mean()) < 0.012
        assert abs(row.var() - 1) < 0.015
        assert abs(stats.kurtosis(row, fisher=False) - 3) < 0.06
        assert stats.kstest(row, "norm").pvalue > 1e-4
    c = np.corrcoef(z)
    assert np.abs(c - np.eye(4)).max() < 0.012


def test_uniform_law_draws():
    lat = oracle.make_lattice(3, 0.25)
    u = oracle.noise_draws(lat, seed=1, t=0, sites=np.arange(100_000), law="uniform")
    assert u.shape == (6, 100_000)
    for row in u:
        assert stats.kstest(row, "uniform").pvalue > 1e-4


def test_block_assignment_d3q7():
    # moments 1..4 use block 0 words 0..3, moments 5..6 block 1 words 0..1
    lat = oracle.make_lattice(3, 0.25)
    u = oracle.noise_draws(lat, seed=3, t=9, sites=np.arange(8), law="uniform")
    r0 = philox.philox4x32_10(np.arange(8), 0, 9, 0, 3, 0)
    r1 = philox.philox4x32_10(np.arange(8), 0, 9, 1, 3, 0)
    exp = [philox.words_to_uniform(x) for x in list(r0) + list(r1)[:2]]
    assert np.array_equal(u, np.array(exp))


def test_site_high_word_used():
    lat = oracle.make_lattice(1)
    big = np.array([5, 5 + (1 << 32)], dtype=np.uint64)
    u = oracle.noise_draws(lat, seed=0, t=0, sites=big, law="uniform")
    assert u[0, 0] != u[0, 1]


def test_step_wraps_mod_2_32():
    lat = oracle.make_lattice(1)
    a = oracle.noise_draws(lat, 0, 3, np.arange(4))
    b = oracle.noise_draws(lat, 0, 3 + (1 << 32), np.arange(4))
    assert np.array_equal(a, b)
