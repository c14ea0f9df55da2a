"""Pins of the oracle's lattice constants against what the paper fixes."""

import json
import math
import os

import numpy as np
import pytest

import oracle

THETAS = {1: [1 / 3, 0.2, 0.7], 2: [1 / 3, 0.2, 0.45], 3: [0.25, 1 / 6, 0.3]}


def _eval(expr, theta):
    return eval(expr, {"__builtins__": {}}, {"sqrt": math.sqrt, "theta": theta})


@pytest.mark.parametrize("d", [1, 2, 3])
def test_weights_meet_equilibrium_moments(d):
    # Sec. II, eqs. (f0_0)-(f0_2): sum w = 1, sum w v = 0, sum w v v = theta delta.
    for th in THETAS[d]:
        lat = oracle.make_lattice(d, th)
        v = lat.v.astype(float)
        assert abs(lat.w.sum() - 1.0) < 1e-15
        assert np.abs(lat.w @ v).max() < 1e-15
        second = np.einsum("i,ia,ib->ab", lat.w, v, v)
        assert np.abs(second - th * np.eye(d)).max() < 1e-15
        # the D2Q5 weights printed in Sec. II, and their 1-D / 3-D analogues
        assert abs(lat.w[0] - (1 - d * th)) < 1e-15
        assert np.abs(lat.w[1:] - th / 2).max() < 1e-15


def test_d2q5_basis_is_the_printed_matrix(golden_dir):
    with open(os.path.join(golden_dir, "d2q5_moment_matrix.json")) as fh:
        rows = json.load(fh)["rows"]
    for th in THETAS[2]:
        lat = oracle.make_lattice(2, th)
        printed = np.array([[_eval(e, th) for e in r] for r in rows])
        assert np.abs(lat.m - printed).max() < 1e-14


@pytest.mark.parametrize("d", [1, 2, 3])
def test_basis_orthonormal_complete(d):
    for th in THETAS[d]:
        lat = oracle.make_lattice(d, th)
        Q = lat.Q
        G = lat.m @ np.diag(lat.w) @ lat.m.T             # <m^a m^b>_M = delta^ab
        assert np.abs(G - np.eye(Q)).max() < 1e-14
        assert np.abs(lat.n @ lat.m.T - np.eye(Q)).max() < 1e-14   # sum_i n_i^a m_i^b
        assert np.abs(lat.m.T @ lat.n - np.eye(Q)).max() < 1e-14   # sum_a m_i^a n_j^a
        # sum_i m_i^a w_i = delta^{a0} (Sec. II, equilibrium moments)
        e0 = np.zeros(Q)
        e0[0] = 1
        assert np.abs(lat.m @ lat.w - e0).max() < 1e-14
        assert np.abs(lat.m[0] - 1.0).max() < 1e-15


@pytest.mark.parametrize("d", [1, 2, 3])
def test_velocity_is_scaled_current_moment(d):
    # Sec. III: v_{i alpha} = sqrt(theta) m_i^{alpha+1}
    for th in THETAS[d]:
        lat = oracle.make_lattice(d, th)
        for a in range(d):
            assert np.abs(lat.v[:, a] - math.sqrt(th) * lat.m[1 + a]).max() < 1e-14


def test_d2q5_second_moment_decomposition():
    # Sec. III: v_x v_x = theta (m^0 + sqrt(1/(2 theta)) m^n + sqrt((1-2 theta)/(2 theta)) m^s),
    # where the paper labels the last two rows m^4, m^5 (rows 3 and 4 of the matrix).
    for th in THETAS[2]:
        lat = oracle.make_lattice(2, th)
        vx2 = lat.v[:, 0].astype(float) ** 2
        rhs = th * (lat.m[0] + math.sqrt(1 / (2 * th)) * lat.m[3]
                    + math.sqrt((1 - 2 * th) / (2 * th)) * lat.m[4])
        assert np.abs(vx2 - rhs).max() < 1e-14


def test_d3q7_traceless_pair_and_classes():
    lat = oracle.make_lattice(3, 0.25)
    th = 0.25
    assert np.allclose(lat.m[4], np.array([0, 1, 1, -1, -1, 0, 0]) / math.sqrt(2 * th))
    assert np.allclose(lat.m[5], np.array([0, 1, 1, 1, 1, -2, -2]) / math.sqrt(6 * th))
    assert lat.cls == (0, 1, 1, 1, 2, 2, 3)
    assert oracle.make_lattice(2).cls == (0, 1, 1, 2, 3)
    assert oracle.make_lattice(1).cls == (0, 1, 3)


def test_theta_validation():
    with pytest.raises(ValueError):
        oracle.make_lattice(3, 1 / 3)
    with pytest.raises(ValueError):
        oracle.make_lattice(2, 0.0)
