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
* Sec. IV, Fourier sums of the populations with the paper's sign,
  f_i(k, t) = sum_x exp(+2 pi i k.x / L) f_i(x, t), the population structure
  factor S_ij(k) = <f_i(k, t) f_j(-k, t)> (eqs. fkfk, FourierTest) and, in the
  equilibrium-dynamics part, the time correlator <rho(k, 0) rho(-k, t)>
  (eq. TimeCorrEqn).  For real fields f(-k) is the complex conjugate of f(k).
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


def population_amplitudes(f, kvecs, method="direct"):
    """Fourier sums of every population with the paper's sign (Sec. IV):
    a[n, i] = sum_x exp(+2 pi i sum_a k_a x_a / L_a) f_i(x) for k = kvecs[n].

    f is (Q, *dims) with x fastest; kvecs is (nk, d).  Returns complex (nk, Q).
    method "direct" evaluates the sum as written; "fft" reads numpy's FFT,
    whose kernel has the opposite sign, at -k.  Pinned by: direct == fft, a
    single occupied site giving the pure phase, sum_i a_i(0) = total mass, and
    Parseval (sum over all k of a_i(k) conj(a_j(k)) = N sum_x f_i f_j)."""
    f = np.asarray(f, dtype=np.float64)
    Q = f.shape[0]
    d = f.ndim - 1
    shape = f.shape[1:]
    L = shape[::-1]
    kvecs = np.asarray(kvecs, dtype=np.int64).reshape(-1, d)
    out = np.empty((len(kvecs), Q), dtype=np.complex128)
    if method == "fft":
        F = np.fft.fftn(f, axes=tuple(range(1, d + 1)))
        for n, k in enumerate(kvecs):
            idx = tuple(int(-k[ax]) % L[ax] for ax in reversed(range(d)))
            out[n] = F[(slice(None),) + idx]
        return out
    grids = np.meshgrid(*[np.arange(m) for m in shape], indexing="ij")
    coords = grids[::-1]
    for n, k in enumerate(kvecs):
        phase = np.zeros(shape)
        for ax in range(d):
            phase = phase + k[ax] * coords[ax] / L[ax]
        e = np.exp(2j * np.pi * phase)
        for i in range(Q):
            out[n, i] = np.sum(e * f[i])
    return out


def correlate(f0, p, nsteps, kvecs, every, nlag, t0=0, rho_eq=None):
    """Run the oracle for nsteps steps from f0 (step index t0) and accumulate
    the population correlators at every step t with t % every == 0, on the
    state before that step's collision:

      sij[n, i, j] += f_i(k_n, t) f_j(-k_n, t)                 (eq. FourierTest)
      ct[n, l]     += rho(k_n, t_s) rho(-k_n, t_{s+l}),  l < nlag  (eq. TimeCorrEqn)

    where t_s is the s-th sampled step and rho(k) = sum_i f_i(k).  The lag-l
    sum has (nsamples - l) terms.  Returns a dict of the complex sums, the
    number of samples and the final state."""
    from .step import run, mean_density
    lat = p.lattice()
    if p.noise == "global" and rho_eq is None:
        rho_eq = mean_density(f0)
    kvecs = np.asarray(kvecs, dtype=np.int64)
    nk, Q = len(kvecs), lat.Q
    sij = np.zeros((nk, Q, Q), dtype=np.complex128)
    ct = np.zeros((nk, nlag), dtype=np.complex128)
    history = []
    f = np.asarray(f0, dtype=np.float64)
    for t in range(t0, t0 + nsteps):
        if every > 0 and t % every == 0:
            a = population_amplitudes(f, kvecs)
            sij += a[:, :, None] * np.conj(a[:, None, :])
            r = a.sum(axis=1)
            history.append(r)
            s = len(history) - 1
            for l in range(min(nlag, s + 1)):
                ct[:, l] += history[s - l] * np.conj(r)
        f = run(f, p, 1, t0=t, rho_eq=rho_eq, lat=lat)
    return {"sij": sij, "ct": ct, "nsamples": len(history), "f": f}


def profile(f, axis=0):
    """Density profile along one axis (Sec. IV, non-equilibrium dynamics: the
    front is averaged over the other directions): for every coordinate c
    along `axis` (0 = x, 1 = y, 2 = z), the sums over all sites with that
    coordinate of rho and of rho^2.  Returns (sum_rho, sum_rho2), each of the
    axis' length."""
    f = np.asarray(f, dtype=np.float64)
    rho = f.sum(axis=0)                    # index order (.., y, x)
    d = rho.ndim
    keep = d - 1 - axis                    # array axis of the requested lattice axis
    others = tuple(a for a in range(d) if a != keep)
    return rho.sum(axis=others), (rho * rho).sum(axis=others)
