"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the lattice Boltzmann method: it draws
random numbers and builds plain fields.  Anything that depends on the
method (the equilibrium weights, for instance) is passed in by the caller,
which takes it from its own side (the library's constant query on the
product side, the oracle on the test side).

All generators use numpy's PCG64 with an explicit seed, independent of the
Philox noise stream of the method.

Recipes (shapes and value distributions of the paper's workloads):
* equilibrium counts: f_i(x) ~ Poisson(lam_i) i.i.d., with lam_i = rho_mean w_i
  supplied by the caller (the ideal-gas occupation statistics of Sec. II);
* sine mode: rho(x) = rho_mean (1 + a sin(2 pi x / Lx));
* Gaussian random field: rho(x) = rho_mean + sigma z(x), z ~ N(0, 1) i.i.d.;
* step profile: rho = rho_hi on 0.25 Lx <= x < 0.75 Lx and rho_lo elsewhere
  (the diffusion-front initial condition of Sec. IV);
* ensembles and request streams for the batched and served workloads.
"""

import math

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def array_shape(dims):
    """numpy shape (.., Ny, Nx) of a lattice with sizes dims = (Nx[, Ny[, Nz]])."""
    return tuple(int(n) for n in reversed(tuple(dims)))


def poisson_counts(dims, lam, seed=0):
    """Independent Poisson counts, one array per mean: shape (Q, *shape)."""
    g = rng(seed)
    shape = array_shape(dims)
    lam = np.asarray(lam, dtype=np.float64)
    return np.stack([g.poisson(l, size=shape).astype(np.float64) for l in lam])


def sine_field(dims, mean, amplitude=0.1, axis=0):
    """mean * (1 + amplitude * sin(2 pi x_axis / L_axis))."""
    shape = array_shape(dims)
    L = int(dims[axis])
    x = np.arange(L, dtype=np.float64)
    prof = mean * (1.0 + amplitude * np.sin(2.0 * math.pi * x / L))
    view = [1] * len(shape)
    view[len(shape) - 1 - axis] = L
    return np.broadcast_to(prof.reshape(view), shape).copy()


def gaussian_field(dims, mean, sigma, seed=0):
    g = rng(seed)
    return mean + sigma * g.standard_normal(array_shape(dims))


def step_field(dims, rho_hi, rho_lo):
    shape = array_shape(dims)
    Lx = int(dims[0])
    x = np.arange(Lx)
    prof = np.where((x >= 0.25 * Lx) & (x < 0.75 * Lx), rho_hi, rho_lo).astype(np.float64)
    return np.broadcast_to(prof, shape).copy()


def outer(vec, field):
    """vec[i] * field for every i: shape (len(vec), *field.shape)."""
    vec = np.asarray(vec, dtype=np.float64)
    return vec.reshape((-1,) + (1,) * field.ndim) * field[None]


def ensemble(n1, n2, seed=0, L1=(64, 4096), L2=(128, 1024), omega=(0.5, 1.9),
             rho=(0.1, 100.0), base_seed=1000):
    """Replica descriptions of the batched workload: n1 one-dimensional
    replicas with L ~ U{L1}, then n2 two-dimensional replicas with
    independent sides ~ U{L2}; omega ~ U[omega], mean density log-uniform in
    rho, Philox seed base_seed + r."""
    g = rng(seed)
    reps = []
    for r in range(n1 + n2):
        d = 1 if r < n1 else 2
        if d == 1:
            dims = (int(g.integers(L1[0], L1[1] + 1)),)
        else:
            dims = (int(g.integers(L2[0], L2[1] + 1)), int(g.integers(L2[0], L2[1] + 1)))
        om = float(g.uniform(*omega))
        rm = float(math.exp(g.uniform(math.log(rho[0]), math.log(rho[1]))))
        reps.append({"d": d, "dims": dims, "omega": om, "rho": rm,
                     "seed": base_seed + r, "init_seed": r})
    return reps


def request_stream(n, rate, seed=0, sites=(1e3, 1e8), steps=(1e2, 1e5),
                   omega=(0.5, 1.9), rho=(0.1, 100.0), models=(1, 2, 3)):
    """n requests with Poisson arrivals at `rate` per second: model uniform
    over `models`, site count and step count log-uniform, square / cubic
    lattices of the nearest side."""
    g = rng(seed)
    t = 0.0
    out = []
    for r in range(n):
        t += float(g.exponential(1.0 / rate))
        d = int(models[int(g.integers(0, len(models)))])
        ns = math.exp(g.uniform(math.log(sites[0]), math.log(sites[1])))
        side = max(3, int(round(ns ** (1.0 / d))))
        nsteps = int(round(math.exp(g.uniform(math.log(steps[0]), math.log(steps[1])))))
        om = float(g.uniform(*omega))
        rm = float(math.exp(g.uniform(math.log(rho[0]), math.log(rho[1]))))
        out.append({"id": r, "arrival": t, "d": d, "dims": (side,) * d,
                    "steps": nsteps, "omega": om, "rho": rm, "seed": r})
    return out


def block_profile(nx, rho_in, rho_out):
    """Density rho_in on [nx/4, 3nx/4), rho_out elsewhere (the step initial
    condition of a diffusion front on a periodic line)."""
    x = np.arange(nx)
    return np.where((x >= nx // 4) & (x < 3 * nx // 4), rho_in, rho_out).astype(np.float64)


def poisson_sites(lam, seed=0):
    """Independent Poisson counts with a mean per entry of lam (any shape)."""
    return rng(seed).poisson(np.asarray(lam, dtype=np.float64)).astype(np.float64)
