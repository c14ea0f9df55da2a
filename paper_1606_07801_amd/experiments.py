"""Equilibrium measurements of the paper's Sec. IV on the GPU path.

Each function runs one lattice with the library's kernels and accumulates
the space-time sums on the device (flb_set_moment_sampling), then forms the
quantities the paper reports:

* ``dij``: eq. (dij) / (dijexp), the normalised equal-time correlation of the
  populations at one site (Table I), here from the sample covariance
  <f_i f_j> - <f_i><f_j> (same expectation as the paper's estimator, whose
  large linear terms it removes);
* ``population_moments``: <f_i> and <f_i f_j> over sites and steps (Fig. 1,
  Table II's first two columns, Fig. 3).

    python -m paper_1606_07801_amd.experiments --table1 3 --steps 300000
"""

import argparse
import json

import numpy as np

from . import flb


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
