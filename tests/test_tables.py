"""The breakpoint tables of the device's double-precision Box-Muller map:
the committed header is what its generator writes, and every entry is the
double nearest the exact value (checked with mpmath when it is installed,
else to within an ulp of the math module)."""

import importlib.util
import math
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1606_07801_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_tables", os.path.join(CSRC, "gen_tables.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_committed_header_is_generated():
    with open(os.path.join(CSRC, "flb_tables.hpp")) as fh:
        assert fh.read() == _gen().header()


def test_entries_are_nearest_doubles():
    g = _gen()
    ln_tab, sc_tab = g.tables()
    assert len(ln_tab) == len(sc_tab) == g.NTAB == 128
    try:
        import mpmath
    except ImportError:
        mpmath = None
    for i, ((inv, lnc), (s, c)) in enumerate(zip(ln_tab, sc_tab)):
        q = g.ln_breakpoint(i)
        assert q == (512 if i == 127 else 257 + 2 * i)
        # breakpoints: the middle of [1/2 + i/256, 1/2 + (i+1)/256), the last its right end
        lo, hi = 0.5 + i / 256, 0.5 + (i + 1) / 256
        assert lo < q / 512 <= hi
        assert inv == 2.0 ** -24 / (q / 512)          # a power of two over an odd integer: exact division
        phi = 2 * math.pi * (2 * i + 1) / 1024
        if mpmath is not None:
            mpmath.mp.dps = 40
            x = 2 * mpmath.pi * (2 * i + 1) / 1024
            assert s == float(mpmath.sin(x)) and c == float(mpmath.cos(x))
            assert lnc == float(mpmath.log(mpmath.mpf(q) / 512))
        else:
            assert abs(s - math.sin(phi)) <= 2 * math.ulp(s)
            assert abs(c - math.cos(phi)) <= 2 * math.ulp(c)
            assert abs(lnc - math.log(q / 512)) <= math.ulp(lnc) + 1e-300
    assert ln_tab[127] == (2.0 ** -24, 0.0)


@pytest.mark.parametrize("x", [0.5, 1.0, 1.5])
def test_decimal_series_against_math(x):
    from decimal import Decimal
    g = _gen()
    s, c = g.sin_cos(Decimal(x))
    assert abs(float(s) - math.sin(x)) <= math.ulp(1.0)
    assert abs(float(c) - math.cos(x)) <= math.ulp(1.0)
    assert abs(float(g.pi()) - math.pi) == 0.0
