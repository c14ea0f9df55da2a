"""Lattice statistics: sums of populations and the density structure factor.

Test infrastructure only (see the package docstring).

* Sec. IV, space-time means: <f_i>_exp averages f_i over sites and steps, and
  eq. (dijexp) averages f_i f_j over sites and steps; here the per-snapshot
  sums sum_x f_i and sum_x f_i f_j are formed, together with the total mass
  sum_x rho (constant, Sec. IV, the total-density identity), sum_x rho^2,
  sum_x max(rho, 0), the number of sites with rho < 0 and a count of
  non-finite populations.
* Sec. IV, Fourier test (eq. fkfk and the k = 0 correction): the density
  structure factor is S(k) = |rho(k)|^2 / N with
  rho(k) = sum_x rho(x) exp(-2 pi i k.x / L); it is flat (= rho^eq) for k != 0
  and equals M_tot^2 / N at k = 0 because mass is conserved.
"""

import numpy as np


def density(f):
    return f.sum(axis=0)


def lattice_sums(f):
    """Dictionary of FP64 sums over all sites of one snapshot f (Q, *dims)."""
    f = np.asarray(f, dtype=np.float64)
    Q = f.shape[0]
    flat = f.reshape(Q, -1)
    finite = np.isfinite(flat)
    rho = flat.sum(axis=0)
    sum_ff = np.empty((Q, Q))
    for i in range(Q):
        for j in range(Q):
            sum_ff[i, j] = np.sum(flat[i] * flat[j])
    return {
        "mass": float(rho.sum()),
        "sum_f": flat.sum(axis=1),
        "sum_ff": sum_ff,
        "sum_rho2": float(np.sum(rho * rho)),
        "sum_rho_pos": float(np.sum(np.maximum(rho, 0.0))),
        "n_negative": int(np.sum(rho < 0.0)),
        "nonfinite": int(np.sum(~finite)),
        "nsite": int(flat.shape[1]),
    }


def structure_factor(rho, kvecs, method="direct"):
    """S(k) = |sum_x rho(x) exp(-2 pi i sum_a k_a x_a / L_a)|^2 / N.

    rho has shape (Nx,), (Ny, Nx) or (Nz, Ny, Nx); kvecs is (nk, d) integer
    wave numbers (k_x[, k_y[, k_z]]).  method "direct" evaluates the sum as
    written; method "fft" reads the same sums off numpy's FFT.
    Pinned by: fft == direct, Parseval (sum_k S(k) = sum_x rho^2), and the
    k = 0 value M^2 / N."""
    rho = np.asarray(rho, dtype=np.float64)
    d = rho.ndim
    L = rho.shape[::-1]                    # (Nx, Ny, Nz)
    N = rho.size
    kvecs = np.asarray(kvecs, dtype=np.int64).reshape(-1, d)
    if method == "fft":
        F = np.fft.fftn(rho)               # index order (kz, ky, kx)
        out = np.empty(len(kvecs))
        for n, k in enumerate(kvecs):
            idx = tuple(int(k[ax]) % L[ax] for ax in reversed(range(d)))
            out[n] = abs(F[idx]) ** 2 / N
        return out
    grids = np.meshgrid(*[np.arange(n) for n in rho.shape], indexing="ij")
    coords = grids[::-1]                   # coords[ax] = x_ax over the array
    out = np.empty(len(kvecs))
    for n, k in enumerate(kvecs):
        phase = np.zeros(rho.shape)
        for ax in range(d):
            phase = phase + k[ax] * coords[ax] / L[ax]
        re = np.sum(rho * np.cos(2 * np.pi * phase))
        im = -np.sum(rho * np.sin(2 * np.pi * phase))
        out[n] = (re * re + im * im) / N
    return out
