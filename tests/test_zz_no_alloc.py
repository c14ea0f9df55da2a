"""flb_profile_noalloc: the density profile with its partial sums in the
library's static scratch (no allocation, no synchronisation) against
flb_profile, through the C ABI, on two calls in a row, the second on a
smaller lattice; and its refusal of sizes beyond the scratch."""

import numpy as np
import pytest

from paper_1606_07801_amd import flb
from tests.gpu_common import gpu_lattice, poisson_state

pytestmark = pytest.mark.gpu


def _both(L, axis):
    import torch
    n = L.dims[axis]
    a = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    b = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    L.profile_noalloc(axis, a, b)
    L.sync()
    s, s2 = L.profile(axis)
    return a.cpu().numpy(), b.cpu().numpy(), s, s2


def test_noalloc_profile_equals_profile_twice_then_smaller():
    big = gpu_lattice(3, (96, 40, 36), 4, omega=1.3, seed=3)
    big.set_populations(poisson_state(3, (96, 40, 36), 8.0, seed=5).astype(np.float32))
    big.step(3)
    small = gpu_lattice(2, (50, 20), 8, omega=0.8, seed=4)
    small.set_populations(poisson_state(2, (50, 20), 3.0, seed=6))
    small.step(5)
    for L in (big, small):            # the second call's lattice is smaller
        for axis in range(L.d):
            a, b, s, s2 = _both(L, axis)
            # the same kernels in the same order: the same bits
            assert np.array_equal(a, s) and np.array_equal(b, s2), (L.dims, axis)
            assert np.isfinite(a).all() and np.isfinite(b).all()
    big.close()
    small.close()


def test_noalloc_profile_rejects_beyond_scratch():
    import torch
    # axis 0 needs 16 x 64 x 16385 bytes of partials, above 16 MiB
    L = gpu_lattice(2, (16385, 64), 4)
    a = torch.zeros(16385, dtype=torch.float64, device="cuda")
    with pytest.raises(flb.FlbError) as e:
        L.profile_noalloc(0, a, a)
    assert e.value.code == flb.FLB_EINVAL and "scratch" in str(e.value)
    b = torch.zeros(64, dtype=torch.float64, device="cuda")
    L.set_populations(np.ones((5, 64, 16385), dtype=np.float32))
    L.profile_noalloc(1, b, b.clone())  # axis 1 needs 16 x 64 bytes: accepted
    L.sync()
    L.close()
