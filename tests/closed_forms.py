"""Closed forms the paper (or plain mathematics) fixes, used to pin the oracle
and the GPU path.  Nothing here runs the lattice Boltzmann step.

* f-space collision matrix of the moment-space relaxation (Sec. II):
  Lambda_ij = sum_a n_i^a (1/tau^a) m_j^a.
* Noise-off evolution of one Fourier mode (eq. LB with eq. collision, no xi):
  with hat f(k) = sum_x f(x) exp(-i k.x) the step is
  hat f(t+1) = E(k) [I - Lambda (I - w 1^T)] hat f(t),  E = diag(exp(-i k.v_i)),
  and the density amplitude is 1^T hat f.
* All rates one (Sec. IV, equilibrium dynamics): the density obeys the
  explicit scheme rho(x, t+1) = sum_i w_i rho(x - v_i, t), whose Fourier
  factor is 1 - theta (d - sum_a cos(2 pi k_a / L_a)) (the paper's
  expression with its sign and factor-of-two slips corrected).
* f-space noise covariance (Sec. II, the expression for <xi_i xi_j> before the
  moment transform), for a given density.
* Stationary equal-time statistics on a finite periodic lattice with exact
  mass conservation: site covariance rho^eq (w_i delta_ij - w_i w_j / N), so
  d_ij = delta_ij - sqrt(w_i w_j) / N (the finite-size effect the paper
  attributes to mass conservation below Table I).
* Poisson moments (Appendix, eqs. Poisson2 and f3).
* The diffusion front (Sec. IV, non-equilibrium dynamics): a block of density
  rho_in on the sites [L/4, 3L/4) of a periodic line in density rho_out spreads
  as rho_out + (rho_in - rho_out)/2 sum_i [erf((x - a - iL)/(2 sqrt(D t))) -
  erf((x - b - iL)/(2 sqrt(D t)))] with the block edges a = L/4 - 1/2,
  b = 3L/4 - 1/2 (the paper's expression with the offset rho_out restored and
  the edges placed between lattice sites).
"""

import numpy as np


def lambda_f(m, n, omegas):
    """Lambda_ij = sum_a n_i^a omega_a m_j^a  (n[a, i], m[a, j])."""
    return n.T @ np.diag(omegas) @ m


def mode_matrix(w, v, k, L, Lam):
    """One noise-off step of a single Fourier mode k (integer wave numbers)."""
    Q = len(w)
    kv = np.zeros(Q)
    for ax in range(v.shape[1]):
        kv = kv + 2 * np.pi * k[ax] * v[:, ax] / L[ax]
    E = np.diag(np.exp(-1j * kv))
    C = np.eye(Q) - Lam @ (np.eye(Q) - np.outer(w, np.ones(Q)))
    return E @ C


def density_gain(w, v, k, L, Lam, t):
    """Amplitude of the density mode after t steps from f_i = w_i rho_k."""
    T = mode_matrix(w, v, k, L, Lam)
    vec = np.asarray(w, dtype=complex)
    for _ in range(t):
        vec = T @ vec
    return np.sum(vec)


def ftcs_factor(theta, k, L):
    d = len(k)
    return 1.0 - theta * (d - sum(np.cos(2 * np.pi * k[a] / L[a]) for a in range(d)))


def fspace_noise_cov(w, Lam, rho):
    """<xi_i xi_j> = rho [ sum_kl L_ik L_jl (w_k w_l - w_k d_kl)
                         - sum_k L_jk (w_i w_k - w_i d_ik)
                         - sum_l L_il (w_l w_j - w_l d_lj) ]."""
    w = np.asarray(w)
    B = np.outer(w, w) - np.diag(w)          # B_kl = w_k w_l - w_k delta_kl
    return rho * (Lam @ B @ Lam.T - (Lam @ B.T).T - Lam @ B)


def stationary_dij(w, nsite):
    w = np.asarray(w)
    return np.eye(len(w)) - np.sqrt(np.outer(w, w)) / nsite


def poisson_moments(lam):
    return lam, lam * lam + lam, lam ** 3 + 3 * lam ** 2 + lam


def front_profile(L, t, D, rho_in, rho_out, images=5):
    from math import erf, sqrt
    a, b = L // 4 - 0.5, 3 * L // 4 - 0.5
    w = 2 * sqrt(D * t)
    out = np.empty(L)
    for j in range(L):
        acc = 0.0
        for i in range(-images, images + 1):
            acc += erf((j - a - i * L) / w) - erf((j - b - i * L) / w)
        out[j] = rho_out + (rho_in - rho_out) / 2 * acc
    return out
