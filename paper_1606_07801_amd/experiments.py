"""Equilibrium measurements of the paper's Sec. IV on the GPU path.

Each function runs one lattice with the library's kernels and accumulates
the space-time sums on the device (flb_set_moment_sampling), then forms the
quantities the paper reports:

* ``dij``: eq. (dij) / (dijexp), the normalised equal-time correlation of the
  populations at one site (Table I), here from the sample covariance
  <f_i f_j> - <f_i><f_j> (same expectation as the paper's estimator, whose
  large linear terms it removes);
* ``population_moments``: <f_i> and <f_i f_j> over sites and steps (Fig. 1,
  Table II's first two columns, Fig. 3);
* ``density_sweep``: the same as batch means over a list of mean densities,
  with <max(rho, 0)> and the fraction of negative sites (Figs. 1 and 3);
* ``population_distribution``: the histogram and first three moments of f_1
  from the populations read back every step (Fig. 4, Table II).

    python -m paper_1606_07801_amd.experiments --table1 3 --steps 300000
"""

import argparse
import json

import numpy as np

from . import flb, inputs


def _run(side, rho, steps, burn, omega, noise, law, seed, precision, every=1):
    w, _ = flb.constants(2)
    L = flb.Lattice(2, (side, side), precision=precision, omega=omega, seed=seed, noise=noise, law=law)
    dt = np.float32 if precision == 4 else np.float64
    L.set_populations(np.broadcast_to((rho * w)[:, None, None], (5, side, side)).astype(dt).copy())
    L.step(burn)
    L.set_moment_sampling(every)
    L.step(steps)
    sums, n = L.sampled_moments()
    L.set_moment_sampling(0)
    L.close()
    return w, sums, n


def population_moments(side, rho, steps, burn=100, omega=1.0, noise="local", law="uniform", seed=1,
                       precision=8):
    """Means <f_i> and <f_i f_j> over all sites and `steps` sampled steps."""
    w, sums, n = _run(side, rho, steps, burn, omega, noise, law, seed, precision)
    cnt = float(n * side * side)
    return w, sums["sum_f"] / cnt, sums["sum_ff"] / cnt


def dij(side, rho=120.0, steps=300_000, burn=100, omega=1.0, noise="local", law="uniform", seed=1,
        precision=8):
    """d_ij of Table I: (<f_i f_j> - <f_i><f_j>) / (rho^eq sqrt(w_i w_j))."""
    w, mf, mff = population_moments(side, rho, steps, burn, omega, noise, law, seed, precision)
    rho_eq = rho
    cov = mff - np.outer(mf, mf)
    return cov / (rho_eq * np.sqrt(np.outer(w, w)))


def density_sweep(densities, noise="local", law="uniform", omega=1.0, side=32, steps=200_000, batches=20,
                  burn=2000, seed=3, precision=8):
    """Fig. 1 and Fig. 3: for each mean density, batch means over `batches`
    consecutive stretches of `steps` sampled steps of
      f    <f_i>                 (mean over sites and steps, per population)
      ff   <f_i f_i>             (same-site second moments, per population)
      pos  <max(rho, 0)>         (the mean noise density of local noise)
      neg  fraction of sites with rho < 0
    as arrays (len(densities), batches, ...).  The lattice starts from
    f = w rho and is run `burn` steps first."""
    w, _ = flb.constants(2)
    N = side * side
    per = steps // batches
    out = {"f": [], "ff": [], "pos": [], "neg": []}
    dt = np.float32 if precision == 4 else np.float64
    for rho in densities:
        L = flb.Lattice(2, (side, side), precision=precision, omega=omega, seed=seed, noise=noise, law=law)
        L.set_populations(np.broadcast_to((rho * w)[:, None, None], (5, side, side)).astype(dt).copy())
        L.step(burn)
        L.set_moment_sampling(1)
        prev, prev_n = None, 0
        rows = {k: [] for k in out}
        for _ in range(batches):
            L.step(per)
            sums, n = L.sampled_moments()
            cur = {"f": sums["sum_f"], "ff": np.diag(sums["sum_ff"]), "pos": sums["sum_rho_pos"],
                   "neg": float(sums["n_negative"])}
            cnt = float((n - prev_n) * N)
            for k in out:
                rows[k].append((cur[k] - (prev[k] if prev else 0)) / cnt)
            prev, prev_n = cur, n
        L.close()
        for k in out:
            out[k].append(np.array(rows[k]))
    return w, {k: np.array(v) for k, v in out.items()}


def population_distribution(side, rho, steps, edges, burn=300, batches=10, omega=1.0, noise="local",
                            law="uniform", seed=5, precision=8):
    """Table II (all three columns) and Fig. 4: the distribution of f_1 over
    all sites, read back after each of `steps` steps.  Returns
      m      per-batch means of f_1, f_1^2, f_1^3, shape (batches, 3)
      hist   counts of f_1 in the bins `edges` (values outside the range are
             counted in under / over)
      zero   the number of samples with f_1 exactly 0
    The lattice starts from f = w rho and is run `burn` steps first."""
    w, _ = flb.constants(2)
    L = flb.Lattice(2, (side, side), precision=precision, omega=omega, seed=seed, noise=noise, law=law)
    dt = np.float32 if precision == 4 else np.float64
    L.set_populations(np.broadcast_to((rho * w)[:, None, None], (5, side, side)).astype(dt).copy())
    L.step(burn)
    edges = np.asarray(edges, dtype=np.float64)
    hist = np.zeros(len(edges) - 1, dtype=np.int64)
    under = over = zero = 0
    per = steps // batches
    m = np.zeros((batches, 3))
    for b in range(batches):
        acc = np.zeros(3)
        for _ in range(per):
            L.step(1)
            f1 = L.get_populations()[1].astype(np.float64).ravel()
            f2 = f1 * f1
            acc += (f1.sum(), f2.sum(), (f2 * f1).sum())
            hist += np.histogram(f1, edges)[0]
            under += int((f1 < edges[0]).sum())
            over += int((f1 > edges[-1]).sum())
            zero += int((f1 == 0).sum())
        m[b] = acc / (per * f1.size)
    L.close()
    return {"w": w, "m": m, "hist": hist, "under": under, "over": over, "zero": zero,
            "samples": batches * per * side * side}


def front_initial(nx, ny, rho_in, rho_out, seed=0):
    """Sec. IV, non-equilibrium dynamics: a block of density rho_in between
    0.25 nx and 0.75 nx in density rho_out, uniform in y, as independent
    Poisson counts f_i ~ Poisson(w_i rho(x)) (D2Q5)."""
    w, _ = flb.constants(2)
    rho0 = inputs.block_profile(nx, rho_in, rho_out)
    lam = w[:, None, None] * np.broadcast_to(rho0[None, :], (ny, nx))[None]
    return inputs.poisson_sites(lam, seed)


def diffusion_front(nx=100, ny=10_000, rho_in=20.0, rho_out=120.0, times=(100, 400, 1600), omega=1.0,
                    noise="local", seed=3, precision=8, f0=None):
    """Run the front and return, at each time, the y-averaged density and
    its variance over y for every x (the paper's Figs. 8 and 9)."""
    if f0 is None:
        f0 = front_initial(nx, ny, rho_in, rho_out, seed)
    dt = np.float32 if precision == 4 else np.float64
    L = flb.Lattice(2, (nx, ny), precision=precision, omega=omega, seed=seed, noise=noise)
    L.set_populations(np.ascontiguousarray(f0, dtype=dt))
    out = {"times": list(times), "mean": [], "var": []}
    for t in times:
        L.step(t - L.t)
        s, s2 = L.profile(0)
        m = s / ny
        out["mean"].append(m)
        out["var"].append(s2 / ny - m * m)
    L.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--table1", type=int, default=3, help="lattice side")
    ap.add_argument("--steps", type=int, default=300_000)
    ap.add_argument("--law", default="uniform")
    ap.add_argument("--noise", default="local")
    args = ap.parse_args()
    d = dij(args.table1, steps=args.steps, law=args.law, noise=args.noise)
    print(json.dumps({"side": args.table1, "steps": args.steps, "dij": np.round(d, 6).tolist()}))


if __name__ == "__main__":
    main()
