"""The paper's equilibrium measurements reproduced on the GPU path, with the
paper's own noise law (flat, Sec. IV): Table I (finite-size d_ij on 3x3) and
the first two columns of Table II (low-density population moments).  The
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
