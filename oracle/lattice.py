"""Velocity sets, equilibrium weights and the orthonormal moment basis.

Test infrastructure only (see the package docstring).

Paper passages followed
-----------------------
* Sec. II, equilibrium moment conditions (eqs. f0_0 .. f0_2): the local
  equilibrium carries density rho, zero first moment and second moment
  rho*theta*delta_ab.
* Sec. II, D2Q5 velocity set and eq. (f0def): f_i^0 = rho * w_i with
  w_0 = 1 - 2 theta, w_1..4 = theta / 2.  The paper notes that the one- and
  three-dimensional models follow the same derivation; their weights are the
  unique solution of the same three moment conditions on the D1Q3 and D3Q7
  velocity sets (w_0 = 1 - d theta, w_i = theta / 2).
* Sec. II, moment basis: rows m^a are obtained by Gram-Schmidt
  orthonormalisation of physically relevant seed vectors under the scalar
  product <m^a m^b>_M = sum_i m_i^a w_i m_i^b = delta^ab, with the
  back-transform n_i^a = m_i^a w_i.  For D2Q5 the seeds are
  1, v_x, v_y, v_x^2 - v_y^2, v_x^2 + v_y^2 and the result is the printed
  5x5 matrix.  For D1Q3 the seeds are 1, v_x, v_x^2; for D3Q7 they are
  1, v_x, v_y, v_z, v_x^2 - v_y^2, v_x^2 + v_y^2 - 2 v_z^2, |v|^2 (a fixed
  choice of the traceless pair, which the paper leaves open).
* Sec. III (hydrodynamic limit): isotropy groups the relaxation rates into
  classes rho, j (currents), n (traceless second moments), s (trace).

Velocity order (x is the fastest array axis):
  D1Q3: 0, +x, -x
  D2Q5: 0, +x, -x, +y, -y          (the paper's order)
  D3Q7: 0, +x, -x, +y, -y, +z, -z
"""

from dataclasses import dataclass

import numpy as np

RHO, J, N, S = 0, 1, 2, 3  # relaxation classes


@dataclass(frozen=True)
class Lattice:
    name: str
    d: int               # spatial dimension
    theta: float         # lattice "temperature" theta
    v: np.ndarray        # (Q, d) integer velocities
    w: np.ndarray        # (Q,) equilibrium weights
    m: np.ndarray        # (Q, Q) rows m^a (moment index a, population index i)
    n: np.ndarray        # (Q, Q) back-transform, n[a, i] = n_i^a = m_i^a w_i
    cls: tuple           # relaxation class of each moment row

    @property
    def Q(self):
        return self.v.shape[0]


def _velocities(d):
    vs = [[0] * d]
    for ax in range(d):
        for sgn in (+1, -1):
            e = [0] * d
            e[ax] = sgn
            vs.append(e)
    return np.array(vs, dtype=np.int64)


def _weights(v, theta):
    """Equilibrium weights: w_0 = 1 - d theta, w_i = theta / 2 (Sec. II prints
    these for D2Q5; the same three moment conditions on the D1Q3 and D3Q7
    velocity sets give the analogues with d = 1, 3)."""
    Q, d = v.shape
    w = np.full(Q, theta / 2.0)
    w[0] = 1.0 - d * theta
    return w


def _seeds(v):
    d = v.shape[1]
    vx = v[:, 0].astype(float)
    one = np.ones(v.shape[0])
    if d == 1:
        return [one, vx, vx * vx], (RHO, J, S)
    vy = v[:, 1].astype(float)
    if d == 2:
        return [one, vx, vy, vx * vx - vy * vy, vx * vx + vy * vy], (RHO, J, J, N, S)
    vz = v[:, 2].astype(float)
    return ([one, vx, vy, vz, vx * vx - vy * vy, vx * vx + vy * vy - 2 * vz * vz,
             vx * vx + vy * vy + vz * vz], (RHO, J, J, J, N, N, S))


def _gram_schmidt(seeds, w):
    """Classical Gram-Schmidt under <a, b> = sum_i a_i w_i b_i.  The first
    seed is the conserved row m^0 = (1, .., 1), already of unit norm because
    the weights sum to one; it is kept exactly as the paper prints it."""
    basis = [np.array(seeds[0], dtype=float)]
    for s in seeds[1:]:
        u = np.array(s, dtype=float)
        for b in basis:
            u = u - np.sum(u * w * b) * b
        norm = np.sqrt(np.sum(u * w * u))
        basis.append(u / norm)
    return np.array(basis)


_NAMES = {1: "D1Q3", 2: "D2Q5", 3: "D3Q7"}


def make_lattice(d, theta=None):
    """Build the D1Q3 (d=1), D2Q5 (d=2) or D3Q7 (d=3) lattice.

    theta defaults to 1/3 for D1Q3 and D2Q5 (the paper's simulations) and to
    1/4 for D3Q7, where theta = 1/3 would make the rest weight vanish.
    theta must satisfy 0 < theta < 1/d so that every weight is positive.
    """
    if d not in _NAMES:
        raise ValueError("d must be 1, 2 or 3")
    if theta is None:
        theta = 0.25 if d == 3 else 1.0 / 3.0
    if not (0.0 < theta < 1.0 / d):
        raise ValueError("theta must lie in (0, 1/d)")
    v = _velocities(d)
    w = _weights(v, theta)
    seeds, cls = _seeds(v)
    m = _gram_schmidt(seeds, w)
    n = m * w[None, :]
    return Lattice(_NAMES[d], d, float(theta), v, w, m, n, cls)
