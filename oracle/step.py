"""One time step of the fluctuating lattice Boltzmann method for diffusion.

Test infrastructure only (see the package docstring).

The state is the set of pre-collision populations f_i(x, t), stored as an
array of shape (Q, Nx) / (Q, Ny, Nx) / (Q, Nz, Ny, Nx) with x fastest and
periodic boundaries.  One step is (Sec. II):

  eq. (LB)         f_i(x + v_i, t + 1) = f_i(x, t) + Omega_i
  eq. (collision)  Omega_i = sum_j Lambda_ij (f_j^0 - f_j) + xi_i

carried out in moment space, where the collision matrix is diagonal
(Sec. II, Lambda^ab = delta^ab / tau^a):

  rho     = sum_i f_i                              (the conserved density)
  M^a     = sum_i m_i^a f_i
  f_i^0   = rho w_i                                eq. (f0def)
  M^{a,0} = sum_i m_i^a f_i^0 = rho delta^{a0}     (Sec. II, equilibrium moments)
  M^a*    = M^a + (M^{a,0} - M^a) / tau^a + xi^a
  f_i*    = sum_a n_i^a M^a*,  n_i^a = m_i^a w_i
  f_i(x + v_i, t + 1) = f_i*(x)

with noise of zero mean and variance (eqs. xiglobal / xilocal)

  <xi^a xi^b> = rho_n (2 tau^a - 1) / (tau^a)^2 (1 - delta^{a0} delta^{b0}) delta^ab

where rho_n is the site's density (local noise), the global mean density
rho^eq (global noise), or 0 (noise off).  A negative local density is
treated as zero (Sec. IV, the paragraph closing the algorithm).

Readings of the paper taken here (each is listed in the design notes):
* the noise law is Gaussian by default; the paper's own flat law
  xi^a ~ U(-d^a, d^a), d^a = sqrt(3 var^a) (Sec. IV) is an option;
* one relaxation rate omega = 1/tau per isotropy class (rho, j, n, s); the
  rho class is irrelevant because M^{0,0} = M^0;
* variates come from Philox4x32-10 keyed by the 64-bit seed, with counter
  (site low word, site high word, step modulo 2^32, block), block =
  floor((a - 1) / 4); moment a >= 1 takes variate (a - 1) mod 4 of its
  block; the site index is x + Nx (y + Ny z) of the colliding site and the
  step is the number of steps completed before this collision.
"""

from dataclasses import dataclass

import numpy as np

from .lattice import RHO, J, N, S, make_lattice
from .philox import philox4x32_10, words_to_uniform, box_muller

_NOISE = ("local", "global", "off")
_LAWS = ("gauss", "uniform")


@dataclass
class Params:
    d: int = 2
    theta: float = None          # None -> 1/3 (d = 1, 2) or 1/4 (d = 3)
    omega_j: float = 1.0         # 1 / tau^j (sets D = (tau^j - 1/2) theta)
    omega_n: float = 0.0         # 0 -> omega_j
    omega_s: float = 0.0         # 0 -> omega_j
    seed: int = 0
    noise: str = "local"
    law: str = "gauss"

    def lattice(self):
        return make_lattice(self.d, self.theta)

    def omegas(self, lat):
        """Relaxation rate 1/tau^a of every moment row."""
        om = {RHO: self.omega_j, J: self.omega_j,
              N: self.omega_n or self.omega_j, S: self.omega_s or self.omega_j}
        return np.array([om[c] for c in lat.cls], dtype=np.float64)


def noise_draws(lat, seed, t, sites, law="gauss"):
    """Variates for moments a = 1..Q-1 at the given flat site indices.

    Returns an array (Q-1, K): standard normals for law "gauss", uniforms in
    (0, 1) for law "uniform".  Parity: the Philox words are pinned against an
    independent implementation; the normals by distribution tests."""
    sites = np.asarray(sites, dtype=np.uint64)
    Q = lat.Q
    nblk = (Q - 1 + 3) // 4
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    k0, k1 = seed & 0xFFFFFFFF, seed >> 32
    s_lo = sites & np.uint64(0xFFFFFFFF)
    s_hi = sites >> np.uint64(32)
    out = []
    for b in range(nblk):
        r = philox4x32_10(s_lo, s_hi, int(t) & 0xFFFFFFFF, b, k0, k1)
        u = [words_to_uniform(x) for x in r]
        if law == "gauss":
            z0, z1 = box_muller(u[0], u[1])
            z2, z3 = box_muller(u[2], u[3])
            out.extend([z0, z1, z2, z3])
        else:
            out.extend(u)
    return np.array(out[:Q - 1])


def collide(f, site_idx, lat, p, t, rho_eq=None):
    """Post-collision populations f_i* for populations f of shape (Q, K)
    belonging to the flat site indices site_idx (K,), at step t."""
    if p.noise not in _NOISE or p.law not in _LAWS:
        raise ValueError("unknown noise mode or law")
    f = np.asarray(f, dtype=np.float64)
    rho = f.sum(axis=0)                                  # rho = sum_i f_i
    M = np.tensordot(lat.m, f, axes=(1, 0))              # M^a = sum_i m_i^a f_i
    # M^{a,0} = sum_i m_i^a f_i^0 with f_i^0 = rho w_i (eq. f0def); Sec. II
    # evaluates it in closed form, M^{a,0} = rho delta^{a0}, which is used
    # here so that the conserved moment is not perturbed by rounding
    M0 = np.zeros_like(M)
    M0[0] = rho
    tau = 1.0 / p.omegas(lat)                            # Lambda^ab = delta^ab / tau^a
    var_coef = (2.0 * tau - 1.0) / tau ** 2
    var_coef[0] = 0.0                                    # no noise on the conserved mode
    if p.noise == "local":
        rho_n = np.maximum(rho, 0.0)                     # negative density -> zero
    elif p.noise == "global":
        if rho_eq is None:
            raise ValueError("global noise needs rho_eq")
        rho_n = np.full_like(rho, float(rho_eq))
    else:
        rho_n = np.zeros_like(rho)
    var = var_coef[:, None] * rho_n[None, :]             # <xi^a xi^a>
    xi = np.zeros_like(M)
    if p.noise != "off":
        draws = noise_draws(lat, p.seed, t, site_idx, p.law)
        if p.law == "gauss":
            xi[1:] = np.sqrt(var[1:]) * draws
        else:
            d = np.sqrt(3.0 * var[1:])                   # flat law on (-d, d)
            xi[1:] = d * (2.0 * draws - 1.0)
    Mstar = M + (M0 - M) / tau[:, None] + xi
    return np.tensordot(lat.n, Mstar, axes=(0, 0))       # f_i* = sum_a n_i^a M^a*


def _dims(f):
    return f.shape[1:]


def stream(fstar, lat):
    """f_i(x + v_i) = f_i*(x) on the periodic lattice (eq. LB)."""
    out = np.empty_like(fstar)
    d = lat.d
    for i in range(lat.Q):
        shift = tuple(int(lat.v[i, ax]) for ax in range(d))
        axes = tuple(-1 - ax for ax in range(d))        # x is the last axis
        out[i] = np.roll(fstar[i], shift, axis=axes)
    return out


def step(f, lat, p, t, rho_eq=None):
    """One full step t -> t + 1 of the lattice f (Q, *dims)."""
    Q = lat.Q
    dims = _dims(f)
    nsite = int(np.prod(dims))
    flat = f.reshape(Q, nsite)
    fstar = collide(flat, np.arange(nsite, dtype=np.uint64), lat, p, t, rho_eq)
    return stream(fstar.reshape((Q,) + dims), lat)


def mean_density(f):
    Q = f.shape[0]
    return float(f.sum()) / (f.size // Q)


def run(f, p, nsteps, t0=0, rho_eq=None, lat=None):
    """Advance f by nsteps steps starting at step index t0.  For global noise
    rho^eq defaults to the mean density of the initial state (mass is
    conserved, so it is the same at every step)."""
    lat = lat or p.lattice()
    if p.noise == "global" and rho_eq is None:
        rho_eq = mean_density(f)
    for t in range(t0, t0 + nsteps):
        f = step(f, lat, p, t, rho_eq)
    return f


def step_sites(f, lat, p, t, coords, rho_eq=None):
    """Post-step populations f_i(x, t + 1) at selected sites only.

    coords is an integer array (K, d) of (x[, y[, z]]) coordinates.  The value
    of population i at x after the step is f_i*(x - v_i), so each population
    collides the site it comes from.  Used to check full-size lattices one
    sampled site at a time.  Returns (Q, K)."""
    Q, d = lat.Q, lat.d
    dims = _dims(f)                     # (.., Ny, Nx)
    L = dims[::-1]                      # (Nx, Ny, Nz)
    coords = np.asarray(coords, dtype=np.int64).reshape(-1, d)
    out = np.empty((Q, coords.shape[0]))
    flat = f.reshape(Q, -1)
    for i in range(Q):
        src = (coords - lat.v[i][None, :]) % np.array(L)[None, :]
        idx = np.zeros(coords.shape[0], dtype=np.int64)
        for ax in reversed(range(d)):
            idx = idx * L[ax] + src[:, ax]
        fs = collide(flat[:, idx], idx.astype(np.uint64), lat, p, t, rho_eq)
        out[i] = fs[i]
    return out


def run_sites(f0, lat, p, t0, nsteps, coords, rho_eq=None, horizon=0):
    """Populations f_i(x, t0 + nsteps) at selected sites, evolved from the
    full initial state f0 at step t0.

    The value at x after T steps depends only on the sites within distance T
    of x, so each selected site is evolved on its own window of side 2T + 1
    (periodic coordinates, true site indices for the noise).  Streaming
    inside a window is non-periodic: whatever wraps in at a window edge is
    wrong, but it moves inward one site per step and does not reach the
    centre within T steps.  Returns (Q, K).  Parity: pinned to step() on
    lattices small enough for both."""
    Q, d = lat.Q, lat.d
    dims = _dims(f0)
    L = dims[::-1]
    T = int(nsteps)
    coords = np.asarray(coords, dtype=np.int64).reshape(-1, d)
    K = coords.shape[0]
    if T == 0:
        idx = tuple(coords[:, a] for a in reversed(range(d)))
        return np.asarray(f0[(slice(None),) + idx]).astype(np.float64)
    if p.noise == "global" and rho_eq is None:
        rho_eq = float(np.asarray(f0).sum(dtype=np.float64)) / (np.asarray(f0).size // Q)
    side = 2 * T + 1
    offs = np.arange(-T, T + 1)
    # window coordinates per axis: (K, side)
    wc = [(coords[:, a][:, None] + offs[None, :]) % L[a] for a in range(d)]
    # global flat site index of every window point, array order (K, [z,] [y,] x)
    shape = (K,) + (side,) * d
    gidx = np.zeros(shape, dtype=np.int64)
    for a in reversed(range(d)):
        view = [K] + [1] * d
        view[d - a] = side
        gidx = gidx * L[a] + wc[a].reshape(view)
    flat = np.asarray(f0).reshape(Q, -1)
    W = flat[:, gidx.ravel()].astype(np.float64).reshape((Q,) + shape)
    sites = gidx.ravel().astype(np.uint64)
    if horizon:
        # L1 distance of every window point from its centre
        grid = np.meshgrid(*([offs] * d), indexing="ij")
        dist = sum(np.abs(g) for g in grid)
        minrho = np.full(K, np.inf)
    for t in range(t0, t0 + T):
        if horizon and t >= t0 + T - horizon:
            rho = W.sum(axis=0)
            cone = dist <= (t0 + T - t)
            minrho = np.minimum(minrho, np.where(cone[None], np.abs(rho), np.inf).reshape(K, -1).min(axis=1))
        fs = collide(W.reshape(Q, -1), sites, lat, p, t, rho_eq).reshape((Q,) + shape)
        for i in range(Q):
            sh = tuple(int(lat.v[i, ax]) for ax in range(d))
            ax = tuple(-1 - a for a in range(d))
            W[i] = np.roll(fs[i], sh, axis=ax)
    centre = (slice(None), np.arange(K)) + (T,) * d
    if horizon:
        return W[centre], minrho
    return W[centre]


def run_box(f0, lat, p, t0, nsteps, origin, extent, rho_eq=None, horizon=0):
    """Populations f_i(x, t0 + nsteps) on a box of sites, evolved from the
    full initial state f0 at step t0.

    The box holds the sites origin[a] + j, 0 <= j < extent[a], along every
    axis a (x first; periodic coordinates).  As in run_sites, the value at x
    after T steps depends only on the sites within distance T of x, so the
    box is evolved on a window grown by T sites on every side, with the true
    site indices for the noise.  After each step the window loses its
    outermost layer: streaming inside the window is non-periodic, and only
    that layer received values from outside it.  Returns (Q, *box shape in
    array order, x last).

    horizon > 0 also returns, per box site, the smallest |rho| of any
    collision of the last `horizon` steps inside the site's light cone (a
    collision at step t within L1 distance t0 + T - t of it), the sites whose
    recent history passed near rho = 0.

    Parity: pinned to step() (and the light-cone minimum to a brute-force
    evaluation over full-lattice trajectories) on lattices small enough for
    both, boxes wrapping around the periodic edges."""
    Q, d = lat.Q, lat.d
    dims = _dims(f0)
    L = dims[::-1]
    T = int(nsteps)
    origin = [int(o) for o in origin]
    extent = [int(e) for e in extent]
    # window coordinates per axis (x first), periodic
    wc = [(origin[a] - T + np.arange(extent[a] + 2 * T)) % L[a] for a in range(d)]
    W = np.asarray(f0)[(slice(None),) + np.ix_(*[wc[a] for a in reversed(range(d))])].astype(np.float64)
    gidx = np.zeros((1,) * d, dtype=np.int64)
    for a in reversed(range(d)):
        view = [1] * d
        view[d - 1 - a] = wc[a].size
        gidx = gidx * L[a] + wc[a].reshape(view)
    if p.noise == "global" and rho_eq is None:
        rho_eq = mean_density(np.asarray(f0))
    inner = (slice(1, -1),) * d
    A = None
    for t in range(t0, t0 + T):
        shape = W.shape[1:]
        if horizon and t >= t0 + T - horizon:
            a = np.abs(W.sum(axis=0))
            A = a if A is None else np.minimum(A, a)
            # widen by one site (L1 neighbours); outside the window counts as inf
            grown = A.copy()
            for ax in range(d):
                lo = [slice(None)] * d
                hi = [slice(None)] * d
                lo[ax], hi[ax] = slice(0, -1), slice(1, None)
                grown[tuple(lo)] = np.minimum(grown[tuple(lo)], A[tuple(hi)])
                grown[tuple(hi)] = np.minimum(grown[tuple(hi)], A[tuple(lo)])
            A = grown
        sites = np.broadcast_to(gidx, shape).ravel().astype(np.uint64)
        fs = collide(W.reshape(Q, -1), sites, lat, p, t, rho_eq).reshape((Q,) + shape)
        for i in range(Q):
            sh = tuple(int(lat.v[i, ax]) for ax in range(d))
            W[i] = np.roll(fs[i], sh, axis=tuple(-1 - ax for ax in range(d)))
        W = W[(slice(None),) + inner]
        gidx = np.broadcast_to(gidx, shape)[inner]
        if A is not None:
            A = A[inner]
    if horizon:
        return W, (A if A is not None else np.full(W.shape[1:], np.inf))
    return W


def step_regions(f, plist, region, t, rho_eq=None):
    """One step of a lattice whose temperature and rates vary in space (Sec. IV,
    non-homogeneous systems): the sites with region[x] == r collide with the
    weights and basis of plist[r].theta and the rates of plist[r] (eq. f0def
    with the local theta, eq. collision), then all populations stream
    (eq. LB; the velocity set does not depend on theta).  region has the
    lattice's shape (.., y, x); every plist entry has the same d, seed, noise
    and law."""
    Q = f.shape[0]
    dims = _dims(f)
    nsite = int(np.prod(dims))
    flat = np.asarray(f, dtype=np.float64).reshape(Q, nsite)
    reg = np.asarray(region).reshape(nsite)
    fstar = np.empty_like(flat)
    lats = [p.lattice() for p in plist]
    for r, p in enumerate(plist):
        idx = np.flatnonzero(reg == r)
        if idx.size:
            fstar[:, idx] = collide(flat[:, idx], idx.astype(np.uint64), lats[r], p, t, rho_eq)
    return stream(fstar.reshape((Q,) + dims), lats[0])


def run_regions(f, plist, region, nsteps, t0=0, rho_eq=None):
    """nsteps of step_regions from step index t0 (global noise: rho^eq from
    the initial state unless given)."""
    if plist[0].noise == "global" and rho_eq is None:
        rho_eq = mean_density(f)
    for t in range(t0, t0 + nsteps):
        f = step_regions(f, plist, region, t, rho_eq)
    return f
