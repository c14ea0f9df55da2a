"""Philox4x32-10 counter-based generator and the uniform / Gaussian mappings.

Test infrastructure only (see the package docstring).

The paper fixes only the variance of the noise (eqs. xiglobal, xilocal) and
uses a flat law in its own runs (Sec. IV).  It specifies no generator.  The
noise stream used here, and independently by the GPU library, is:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11): a 4x32-bit counter and a 2x32-bit key; each of
  the 10 rounds multiplies counter words 0 and 2 by two fixed 32-bit
  multipliers, takes the high and low halves of the 64-bit products, and
  mixes the high halves with the other two counter words and the key; the
  key advances between rounds by two Weyl increments (the golden ratio and
  sqrt(3) - 1, scaled by 2^32).
* uniform: u = (2 * (r >> 9) + 1) * 2^-24 for a 32-bit word r.  Every u is an
  odd multiple of 2^-24 in (0, 1), exactly representable in float32 and
  float64, and never 0 or 1.
* Gaussian (Box-Muller, 1958): from (u0, u1), R = sqrt(-2 ln u0),
  z0 = R cos(2 pi u1), z1 = R sin(2 pi u1).

All integer arithmetic is done in numpy uint64 on values below 2^32, so that
32 x 32 -> 64-bit products are exact.
"""

import numpy as np

_U32 = np.uint64(0xFFFFFFFF)

# Round multipliers of Philox4x32 (SC'11, Table of Philox parameters).
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
# Weyl key increments: floor(2^32 * (golden ratio - 1)) and
# floor(2^32 * (sqrt(3) - 1)).
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)


def _u64(x):
    return np.asarray(x).astype(np.uint64) & _U32


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on broadcastable arrays of 32-bit counter words
    (c0..c3) under key words (k0, k1).  Returns four uint64 arrays holding
    32-bit results.  Parity: pinned against an independent library
    implementation on the GPU machine and by statistical tests."""
    c0, c1, c2, c3 = _u64(c0), _u64(c1), _u64(c2), _u64(c3)
    k0, k1 = _u64(k0), _u64(k1)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & _U32
            k1 = (k1 + PHILOX_W1) & _U32
        p0 = PHILOX_M0 * c0          # < 2^64, exact
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _U32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _U32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def words_to_uniform(r):
    """u = (2 * (r >> 9) + 1) / 2^24, as float64."""
    r = _u64(r)
    return ((r >> np.uint64(9)) * np.uint64(2) + np.uint64(1)).astype(np.float64) * 2.0 ** -24


def box_muller(u0, u1):
    """Two independent standard normals from two uniforms (Box-Muller)."""
    R = np.sqrt(-2.0 * np.log(u0))
    ang = 2.0 * np.pi * u1
    return R * np.cos(ang), R * np.sin(ang)
