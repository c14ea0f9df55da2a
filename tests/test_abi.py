"""The C-ABI library loads and exports every function include/flb.h declares;
host-side validation works without a GPU (no compute calls here)."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1606_07801_amd import flb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(flb_\w+)\s*\(", src, flags=re.M)
    return names


def test_library_exports_every_declared_symbol():
    lib = flb.load()
    declared = _declared()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(flb.EXPORTS)


def test_api_calls_carry_roctx_ranges():
    # the API calls mark their host-side extent with roctx ranges: the
    # library imports the range API (recorded by rocprofv3 --marker-trace)
    import subprocess
    out = subprocess.run(["nm", "-D", flb.LIB_PATH], capture_output=True, text=True, check=True).stdout
    undefined = {ln.split()[-1] for ln in out.splitlines() if " U " in ln}
    assert {"roctxRangePushA", "roctxRangePop"} <= undefined
    src = open(os.path.join(ROOT, "paper_1606_07801_amd", "csrc", "flb.hip")).read()
    for name in ("flb_step", "flb_set_populations", "flb_get_populations", "flb_structure_factor"):
        assert f'TraceRange trace_("{name}")' in src, name


def test_version_and_constants():
    lib = flb.load()
    assert lib.flb_version() == 1
    for d in (1, 2, 3):
        w, m = flb.constants(d)
        Q = 2 * d + 1
        assert w.shape == (Q,) and m.shape == (Q, Q)
        assert abs(w.sum() - 1) < 1e-15
        assert np.abs(m @ np.diag(w) @ m.T - np.eye(Q)).max() < 1e-14


def test_constants_agree_with_oracle():
    import oracle
    for d in (1, 2, 3):
        for th in ({1: 0.3, 2: 0.2, 3: 0.25}[d], 0.0):
            w, m = flb.constants(d, th)
            lat = oracle.make_lattice(d, th or None)
            assert np.abs(w - lat.w).max() < 1e-15
            assert np.abs(m - lat.m).max() < 1e-14


@pytest.mark.parametrize("bad", [
    dict(model=4), dict(precision=2), dict(theta=0.5), dict(omega=2.0), dict(omega=0.0),
    dict(omega_n=2.5), dict(noise="bogus"), dict(kernel="bogus"), dict(tile_x=100),
    dict(tile_rows=3), dict(dims=(0, 4)),
])
def test_invalid_params_rejected(bad):
    kw = dict(model=2, dims=(8, 8), precision=4)
    kw.update(bad)
    model, dims = kw.pop("model"), kw.pop("dims")
    try:
        p = flb.make_params(model, dims, **kw)
    except KeyError:
        return  # rejected by the binding's name tables
    with pytest.raises(flb.FlbError) as e:
        flb.required_bytes(p)
    assert e.value.code == flb.FLB_EINVAL


def test_required_bytes():
    p = flb.make_params(2, (64, 32), precision=4)
    pop, work = flb.required_bytes(p)
    assert pop == 2 * 5 * 64 * 32 * 4
    assert work > 0
    p3 = flb.make_params(3, (16, 8, 4), precision=8)
    pop3, _ = flb.required_bytes(p3)
    assert pop3 == 2 * 7 * 16 * 8 * 4 * 8


def test_extra_sizes_must_be_one():
    p = flb.make_params(1, (16,), precision=8)
    p.n[1] = 2
    with pytest.raises(flb.FlbError):
        flb.required_bytes(p)


def test_gauss_map_validation_without_gpu():
    lib = flb.load()
    vp = ctypes.c_void_p
    assert lib.flb_gauss_map(3, vp(8), 4, vp(8), None) == flb.FLB_EINVAL
    assert lib.flb_gauss_map(8, vp(8), -1, vp(8), None) == flb.FLB_EINVAL
    assert lib.flb_gauss_map(8, None, 4, vp(8), None) == flb.FLB_EINVAL
    assert lib.flb_gauss_map(4, None, 0, None, None) == 0


def test_sample_size_bounds_without_gpu():
    lib = flb.load()
    vp = ctypes.c_void_p
    assert lib.flb_gauss_map(8, vp(8), 1 << 31, vp(8), None) == flb.FLB_EINVAL
    assert lib.flb_noise_sample(2, 8, 0, 1, 0, 0, 1 << 31, None, None, None) == flb.FLB_EINVAL
    assert lib.flb_noise_sample(2, 8, 0, 1, 0, 0, 0, None, None, None) == 0
