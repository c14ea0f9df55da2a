"""Benchmark of the fluctuating lattice Boltzmann step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Headline workload (one "step" = one pass of the hot path over the lattice):
a D2Q5 lattice of 4096 x 4096 sites, float32 populations, mean density 10
with a sine mode of relative amplitude 0.1 plus equilibrium noise (Poisson
counts f_i ~ Poisson(w_i rho(x))), omega = 1, local Gaussian noise, seed 0;
every step runs the fused stream-collide kernel, and every `--sample-every`
steps (default 10) the sampled variant of the step also accumulates the FP64
density marginals, from which the structure factor of 1024 axis modes is
accumulated on the device; the FP64 lattice sums are taken at the end.

The same line carries, each timed in this run with its oracle error:
the one-step kernel on the same state (depth1), the plain and the tuned
FP64 paths (the comparator), the D3Q7 512^3 FP32 lattice (c3_*) and the
1024 + 256 replica FP32 ensemble (c4_*); and the first 16 requests of the
served stream under an HBM budget with two storage policies (c5_*).
Prints one JSON line.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
# VALU: one wave64 instruction per CU per clock (a 16-lane SIMD takes four
# clocks per full-rate instruction, four SIMDs per CU), 256 CUs at 2.4 GHz.
# SQ_ACTIVE_INST_VALU counts the same four-clock units, two for a
# transcendental, so the same peak bounds it.
PEAK_VALU_G = 256 * 2.4
CSRC = os.path.join(ROOT, "paper_1606_07801_amd", "csrc")
COUNTER_FILES = [os.path.join(ROOT, "profiles", f) for f in
                 ("step_d2q5_4096_fp32_counters.md", "step_d3q7_512_fp32_counters.md",
                  "batch_ensemble_fp32_counters.md")]
# |rho| below which a collision's noise amplitude sqrt(max(rho, 0)) turns the
# rounding of rho into differences above the tolerance: an FP32 difference d
# of rho (~1e-7 of the populations) moves the amplitude by d / (2 sqrt(rho)),
# which reaches 1e-5 of rho_mean w_i up to rho ~ 0.02; FP64 (1e-16, 1e-12)
# only up to ~1e-6.  Sites whose light cone of the last HORIZON steps holds
# such a collision are reported apart.
NEAR_ZERO = {4: 0.05, 8: 1e-3}
HORIZON = 12       # steps of light cone searched for such collisions


def log(msg):
    """Progress line on stderr (the JSON line is the only stdout output)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def source_hash():
    """Hash of every kernel and launch source; counter summaries taken on
    other sources are ignored."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hpp", ".hip")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def counters(kernel, files=None):
    """Per-launch counter figures of `kernel` from the committed summaries
    whose kernel_source_sha256_16 matches the current sources: a dict of
    traffic_bytes_per_launch (HBM bytes, calibrated), valu_wave_insts_per_launch
    (SQ_INSTS_VALU), valu_active_per_launch (SQ_ACTIVE_INST_VALU) and
    valu_busy (SQ_ACTIVE_INST_VALU over 256 CUs x the per-XCD active clocks),
    whichever the summary has.  A summary lists "kernel: <name>" lines each
    followed by "<key>: <value>" lines."""
    cur = source_hash()
    out = {}
    for path in files or COUNTER_FILES:
        try:
            lines = open(path).read().splitlines()
        except OSError:
            continue
        src, k = None, None
        entries = {}
        for line in lines:
            if ":" not in line or line.startswith(("#", "|", " ", "`")):
                continue
            key, v = (x.strip() for x in line.split(":", 1))
            if key == "kernel_source_sha256_16":
                src = v
            elif key == "kernel":
                k = v
            elif k and k == kernel:
                try:
                    entries[key] = float(v)
                except ValueError:
                    pass
        if src == cur and entries:
            out.update(entries)
    return out


def measured_traffic(kernel):
    v = counters(kernel).get("traffic_bytes_per_launch")
    return int(v) if v else None


def roofline(kernel, us, alg_bytes, steps_per_launch, sites):
    """Roofline object of one launch of `kernel` lasting `us` (live, HIP
    events).  alg_bytes: the bytes a launch must move, reading and writing
    every population once (2 Q s N; a two-step pass moves its state once
    for two steps).  The HBM fraction uses the counted bytes when a current
    summary has them, the algorithmic bytes otherwise; the ALU fraction is
    SQ_ACTIVE_INST_VALU per launch over the time against 614.4 G/s.  The
    binding roofline is the larger fraction."""
    c = counters(kernel)
    t = us * 1e-6
    traffic = int(c["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in c else None
    hbm_gbs = (traffic if traffic else alg_bytes) / t / 1e9
    hbm = {"achieved": round(hbm_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(hbm_gbs / PEAK_HBM_GBS, 4), "bytes": "counted" if traffic else "algorithmic"}
    alu = None
    if "valu_active_per_launch" in c:
        a = c["valu_active_per_launch"] / t / 1e9
        alu = {"achieved": round(a, 1), "peak": PEAK_VALU_G, "unit": "G VALU quad-cycles/s",
               "frac": round(a / PEAK_VALU_G, 4)}
        if "valu_wave_insts_per_launch" in c:
            alu["issue_frac"] = round(c["valu_wave_insts_per_launch"] / t / 1e9 / PEAK_VALU_G, 4)
        if "valu_busy" in c:
            alu["busy_frac_profiled"] = c["valu_busy"]
    bind = "alu" if alu and alu["frac"] > hbm["frac"] else "hbm"
    main_ = alu if bind == "alu" else hbm
    r = {"bound": bind, "achieved": main_["achieved"], "peak": main_["peak"], "unit": main_["unit"],
         "frac": main_["frac"], "traffic": traffic, "kernel": kernel, "kernel_us": round(us, 2),
         "bytes_per_launch": alg_bytes, "steps_per_launch": steps_per_launch, "hbm": hbm, "alu": alu}
    flat = {"hbm_frac_measured": hbm["frac"] if traffic else None,
            "valu_frac": alu["frac"] if alu else None,
            "effective_gbs": round(alg_bytes * steps_per_launch / t / 1e9, 1),
            "kernel_mlups": round(steps_per_launch * sites / t / 1e6, 1)}
    return r, flat


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--sample-every", type=int, default=10)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the D3Q7 and ensemble legs")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle checks of the legs")
    ap.add_argument("--no-served", action="store_true", help="skip the served leg")
    ap.add_argument("--requests", type=int, default=48, help="served workload: number of requests")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--workload", default="lattice", choices=["lattice", "d1q3", "d3q7", "batched", "served"],
                    help="lattice: the default line; the others print their own line")
    return ap.parse_args()


def kernel_name(cfg, d=2, prec="float"):
    """Name of the step kernel a launch configuration selects (as profiled)
    for local Gaussian noise (the two-step kernels' instances with that noise
    plan fixed at compile time, plan 1)."""
    nt = "true" if cfg.get("nt_store") else "false"
    if cfg.get("kernel") == "two":
        ty = cfg.get("tile_rows") or 8
        return f"flb::k_step2_d2<{prec}, {2 if ty <= 2 else ty}, {nt}, false, 1>"
    if cfg.get("kernel") == "flat":
        return f"flb::k_step_flat<{d}, {prec}, {cfg.get('tile_rows') or (2 if d == 2 else 1)}, {nt}, 1>"
    if cfg.get("kernel") == "plain":
        return f"flb::k_step_plain<{d}, {prec}>"
    return f"flb::k_step_rows<{d}, {prec}, {cfg.get('tile_rows') or 4}, {nt}>"


def steps_per_launch(cfg):
    """Steps one launch of the dominant step kernel advances."""
    return 2 if cfg.get("kernel") == "two" else 1


def headline_state(torch, flb, n, precision, seed=0):
    """f_i ~ Poisson(w_i rho(x)), rho = 10 (1 + 0.1 sin 2 pi x / n), drawn on
    the device; returned as a device tensor."""
    from paper_1606_07801_amd import inputs
    w, _ = flb.constants(2)
    rho = torch.from_numpy(inputs.sine_field((n, n), 10.0, 0.1)).to("cuda")
    lam = torch.tensor(w, dtype=torch.float64, device="cuda").reshape(-1, 1, 1) * rho[None]
    g = torch.Generator(device="cuda").manual_seed(seed)
    f = torch.poisson(lam, generator=g)
    return f.to(torch.float32 if precision == 4 else torch.float64).contiguous()


def time_steps(torch, L, steps, sample_every, per_launch=1):
    """Run `steps` steps (the lattice samples S(k) itself every
    `sample_every` steps) and return (wall ms per step, mean duration of one
    launch of the dominant step kernel).  Each run of unsampled steps is one
    flb_step call; HIP events on the lattice's stream bracket the part of it
    made of whole launches of the dominant kernel (per_launch steps each),
    which is then divided by their number."""
    st = L.stream
    pairs = []
    t = L.t
    end = t + steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while t < end:
        if sample_every and t % sample_every == 0:
            # the sampled step: alone, or the first of a sampled pair
            k = 2 if per_launch == 2 and t + 1 < end and (t + 1) % sample_every else 1
            L.step(k)
            t += k
            continue
        nxt = min(end, (t // sample_every + 1) * sample_every) if sample_every else end
        run = nxt - t
        whole = run - run % per_launch
        if whole:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            L.step(whole)
            e1.record(st)
            pairs.append((e0, e1, whole // per_launch))
        if run % per_launch:
            L.step(run % per_launch)
        t = nxt
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total = sum(e0.elapsed_time(e1) for e0, e1, _ in pairs)
    launches = sum(k for _, _, k in pairs)
    return (t1 - t0) * 1e3 / steps, (total / launches if launches else float("nan"))


def _coords(dims, n, seed):
    """n random sites plus every corner of the box (periodic wrap)."""
    gen = np.random.default_rng(seed)
    pts = np.stack([gen.integers(0, L, n) for L in dims], axis=1)
    corners = np.array(np.meshgrid(*[[0, L - 1] for L in dims], indexing="ij")).reshape(len(dims), -1).T
    return np.concatenate([corners, pts])


def sampled_error(g, f0, d, omega, steps, rho_mean, nsample=2000, seed=7, t0=0, precision=4):
    """Error of the GPU state g (steps after the seeded state f0 at step t0)
    against the oracle at sampled sites, each evolved on its own window:
    max over all sites, max over the sites whose light cone had no
    collision with |rho| < NEAR_ZERO, and the number of such sites."""
    import oracle
    lat = oracle.make_lattice(d)
    p = oracle.Params(d=d, omega_j=omega, seed=0)
    dims = tuple(reversed(np.asarray(f0).shape[1:]))
    coords = _coords(dims, nsample, seed)
    ref, minrho = oracle.run_sites(f0, lat, p, t0, steps, coords, horizon=min(steps, HORIZON))
    idx = tuple(coords[:, a] for a in reversed(range(d)))
    got = np.asarray(g)[(slice(None),) + idx].astype(np.float64)
    floor = rho_mean * lat.w[:, None]
    err = np.abs(got - ref) / np.maximum(np.abs(ref), floor)
    ok = minrho > NEAR_ZERO[precision]
    return {"max_err": float(err.max()), "max_err_well_conditioned": float(err[:, ok].max()) if ok.any() else None,
            "sites": int(len(coords)), "sites_near_rho0": int((~ok).sum())}


def depth1_reference(torch, flb, f0, dims):
    """The one-step flat kernel on the same lattice (each step reads and
    writes every population once): its duration and rooflines, the
    reference for the two-step pass; and its error against the oracle after
    4 steps of the seeded state at sampled sites."""
    cfg = {"kernel": "flat", "tile_rows": 2, "nt_store": 1}
    L = flb.Lattice(2, dims, precision=4, omega=1.0, seed=0, noise="local", **cfg)
    L.set_populations(f0)
    L.step(20)
    st = L.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    L.step(100)
    e1.record(st)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / 100
    N = dims[0] * dims[1]
    r, flat = roofline(kernel_name(cfg), us, 2 * 5 * 4 * N, 1, N)
    out = {"kernel": r["kernel"], "kernel_us": r["kernel_us"], "hbm": r["hbm"], "alu": r["alu"],
           "traffic": r["traffic"], "effective_gbs": flat["effective_gbs"]}
    return out, L


def fp64_paths(torch, flb, tune, f64, dims, k64, check):
    """The comparator: the plain FP64 single-lattice path, and the tuned
    FP64 path, on the same state; each with its error against the oracle
    (a fresh lattice in the same launch configuration, 4 steps, sampled
    sites)."""
    N = dims[0] * dims[1]
    out = {}
    for tag, cfg in (("fp64_plain", {"kernel": "plain"}), ("fp64_tuned", tune.best_config(2, 8, dims))):
        P = flb.Lattice(2, dims, precision=8, omega=1.0, seed=0, **cfg)
        P.set_populations(f64)
        P.step(20)
        spl = steps_per_launch(cfg)
        ms, kern = time_steps(torch, P, k64, 0, spl)
        r, flat = roofline(kernel_name(cfg, prec="double"), kern * 1e3, 2 * 5 * 8 * N, spl, N)
        res = {"kernel": cfg, "mlups": round(N / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
               "effective_gbs": flat["effective_gbs"], "hbm": r["hbm"], "alu": r["alu"]}
        if check:
            P.set_populations(f64)
            P.step(4)
            res["oracle"] = sampled_error(P.get_populations(), f64.cpu().numpy(), 2, 1.0, 4, 10.0, precision=8)
        P.close()
        out[tag] = res
    return out


def sk_flatness(S, kvecs, n, rho_pos, sample_times, exclude):
    """Flatness of the accumulated S(k) (mean over the samples) against
    <max(rho, 0)>, the stationary value for local noise (the state starts
    in equilibrium around the sine profile): per mode z = (S/rho_pos - 1)/sd,
    with sd the standard deviation of the mean of correlated samples of an
    exponential variable whose autocorrelation at lag dt is lambda(k)^(2 dt)
    (lambda = 1 - theta (2 - cos 2 pi kx/n - cos 2 pi ky/n) at unit rates)."""
    th = 1.0 / 3.0
    ts = np.asarray(sample_times, dtype=np.float64)
    zs, ratio = [], []
    for (kx, ky), s in zip(kvecs, S):
        if (kx, ky) in exclude:
            continue
        lam = 1.0 - th * (2.0 - np.cos(2 * np.pi * kx / n) - np.cos(2 * np.pi * ky / n))
        c = np.abs(lam) ** (2.0 * np.abs(ts[:, None] - ts[None, :]))
        sd = np.sqrt(c.sum()) / len(ts)
        ratio.append(s / rho_pos)
        zs.append((s / rho_pos - 1.0) / sd)
    zs = np.asarray(zs)
    return {"modes": int(len(zs)), "samples": int(len(ts)), "mean_ratio": round(float(np.mean(ratio)), 5),
            "mean_z2": round(float(np.mean(zs ** 2)), 3), "max_abs_z": round(float(np.abs(zs).max()), 2)}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(the lattice would shard by slabs with a one-layer halo exchange per step). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(1)
    import torch
    from paper_1606_07801_amd import flb, inputs, tune

    torch.cuda.set_device(0)
    if args.workload != "lattice":
        out = OTHER[args.workload](torch, flb, inputs, tune, args)
        print(json.dumps(out), flush=True)
        return
    n = args.size
    dims = (n, n)
    N = n * n
    Q = 5
    cfg = tune.best_config(2, 4, dims)
    f0 = headline_state(torch, flb, n, 4)
    # the depth-1 comparator on the same state first: its ~120 steps also
    # bring the GPU out of idle before the timed region
    log("depth-1 reference")
    depth1, D1 = depth1_reference(torch, flb, f0, dims)
    L = flb.Lattice(2, dims, precision=4, omega=1.0, seed=0, noise="local", **cfg)
    # the step counter starts where the timed region begins on a sampling step
    se = args.sample_every
    t0 = (-args.warmup) % se if se else 0
    L.set_populations(f0, step=t0)
    kvecs = [(k, 0) for k in range(1, 513)] + [(0, k) for k in range(1, 513)]
    if se:  # S(k) and the lattice sums (FP64 accumulators) of the state every se steps
        L.set_sampling(se, kvecs)
        L.set_moment_sampling(se)

    # warmup, then the timed region (all hot-path rows: step + sampled stats)
    log(f"headline: D2Q5 {n}^2 fp32 {cfg}, warmup {args.warmup}, timed {args.steps}")
    L.step(args.warmup)
    spl = steps_per_launch(cfg)
    t_start = L.t
    ms_step, kern_ms = time_steps(torch, L, args.steps, se, spl)
    m = L.moments()
    S = L.structure_factor(None, mode="read")[:len(kvecs)] if se else None
    msum, nmom = L.sampled_moments() if se else (None, 0)
    L.close()

    value = N / (ms_step * 1e-3) / 1e6  # MLUPS of the whole job
    rl, flat = roofline(kernel_name(cfg), kern_ms * 1e3, 2 * Q * 4 * N, spl, N)
    out = {
        "metric": "MLUPS", "value": round(value, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"D2Q5 {n}x{n} periodic, fp32 populations, rho=10 sine mode 0.1 plus equilibrium "
                        f"(Poisson) noise, omega=1.0, local Gaussian noise (Philox), S(k) of 1024 axis modes "
                        f"and the lattice sums accumulated every {se} steps",
            "kernel": cfg, "sites": N, "step0": t0,
        },
        "roofline": rl,
        **flat,
        "mass_drift_rel": abs(m["mass"] - m["mass0"]) / m["mass0"],
    }
    if se:
        times = [t - t0 for t in range(t0, t_start + args.steps) if t % se == 0]
        out["sk_flat"] = sk_flatness(S, kvecs, n, m["sum_rho_pos"] / N, times, {(1, 0)})
        # the sampled lattice sums: mean site variance of rho over the samples
        # (Poisson equilibrium: rho-bar; the sine mode adds its own variance)
        out["moment_samples"] = nmom
        if nmom:
            out["mean_var_rho"] = round(msum["sum_rho2"] / (nmom * N) - (msum["mass"] / (nmom * N)) ** 2, 4)

    out["depth1"] = depth1
    f_host = f0.cpu().numpy()
    if not args.no_check:
        D1.set_populations(f0)
        D1.step(4)
        out["depth1"]["oracle"] = sampled_error(D1.get_populations(), f_host, 2, 1.0, 4, 10.0)
    D1.close()

    if not args.no_fp64:
        log("fp64 paths")
        f64 = f0.to(torch.float64)
        out.update(fp64_paths(torch, flb, tune, f64, dims, max(args.steps // 4, 40), not args.no_check))
        del f64

    if not args.no_legs:
        log("D3Q7 512^3 leg")
        c3 = leg_d3q7(torch, flb, tune, args, check=not args.no_check)
        log("ensemble leg")
        c4 = leg_ensemble(torch, flb, inputs, tune, args, check=not args.no_check)
        out["c3_d3q7"] = c3
        out["c4_ensemble"] = c4
        # flat keys (survive a parsed view of the line)
        for k in ("mlups", "ms_per_step", "effective_gbs", "hbm_frac_measured", "valu_frac"):
            out[f"c3_{k}"] = c3.get(k)
            out[f"c4_{k}"] = c4.get(k)
        out["c3_err_vs_oracle"] = (c3.get("oracle") or {}).get("max_err")
        out["c4_err_vs_oracle_rho_ge_5"] = (c4.get("oracle") or {}).get("max_err_rho_ge_5")

    if not args.no_legs and not args.no_served:
        log("served leg")
        c5 = leg_served(torch, flb, args)
        out["c5_served"] = c5
        for pol in ("two", "auto"):
            r = c5.get(pol) or {}
            out[f"c5_{pol}_mlups"] = r.get("mlups")
            out[f"c5_{pol}_p50_latency_s"] = r.get("p50_latency_s")
            out[f"c5_{pol}_p99_latency_s"] = r.get("p99_latency_s")
            out[f"c5_{pol}_mean_resident"] = r.get("mean_resident")

    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - ts) / 10
        out["copy_probe"] = {"bytes_each_way": nb, "gbs_read_plus_write": round(2 * nb / dt / 1e9, 1)}
        del src, dst

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, 4 steps of the full lattice)")
        out["cpu_baseline"] = cpu_baseline(flb, n, f_host, cfg, se, kvecs)
        # the gate (as in the tests): populations out of reach of a collision
        # with |rho| < NEAR_ZERO[4]; the maximum over all populations beside it
        cb = out["cpu_baseline"]
        out["err_vs_oracle"] = cb["gpu_fp32_max_err_well_conditioned"]
        out["err_vs_oracle_all_pops"] = cb["gpu_fp32_max_err_vs_oracle"]
        out["n_pops_near_rho0_reach"] = cb["n_pops_near_rho0_reach"]

    print(json.dumps(out), flush=True)


def cpu_baseline(flb, n, f_host, cfg, se, kvecs):
    """The FP64 oracle (single-threaded numpy) on a bounded sample of the
    same workload: 4 steps of the full lattice from the seeded state.  The
    GPU path in the benchmark's launch configuration and sampling (a sampled
    two-step pass, then an unsampled one) runs the same 4 steps from the same
    state and is compared with it, every population; sites within reach of a
    collision with |rho| < NEAR_ZERO[4] (where the noise amplitude
    sqrt(max(rho, 0)) magnifies the FP32 rounding) during those steps are
    counted apart."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import contextlib

    import oracle

    nsteps = 4
    p = oracle.Params(d=2, omega_j=1.0, seed=0, noise="local")
    lat = p.lattice()
    ctx = threadpool_limits(limits=1) if threadpool_limits else contextlib.nullcontext()
    near = []
    dt = 0.0
    with ctx:
        ref = f_host.astype(np.float64)
        for t in range(nsteps):
            near.append(np.abs(ref.sum(axis=0)) < NEAR_ZERO[4])  # collisions of step t near rho = 0
            ts = time.perf_counter()
            ref = oracle.step(ref, lat, p, t)
            dt += time.perf_counter() - ts
    L = flb.Lattice(2, (n, n), precision=4, omega=1.0, seed=0, noise="local", **cfg)
    L.set_populations(f_host)
    if se:
        L.set_sampling(se, kvecs)
    L.step(nsteps)
    g = L.get_populations()
    L.close()
    floor = (10.0 * lat.w).reshape(-1, 1, 1)
    err = np.abs(g.astype(np.float64) - ref) / np.maximum(np.abs(ref), floor)
    # a deviation at a collision of step t reaches at most nsteps - t sites
    # along each axis by the end: flag every site within that box
    site = np.zeros((n, n), dtype=bool)
    for t, nr in enumerate(near):
        r = nsteps - t
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                site |= np.roll(nr, (dy, dx), axis=(0, 1))
    flag = np.broadcast_to(site, err.shape)
    return {"value": round(nsteps * n * n / dt / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{nsteps} steps of the {n}x{n} D2Q5 lattice from the seeded state ({dt:.1f} s)",
            "gpu_kernel": cfg,
            "gpu_fp32_max_err_vs_oracle": float(err.max()),
            "gpu_fp32_max_err_well_conditioned": float(err[~flag].max()),
            "n_pops_near_rho0_reach": int(flag.sum())}


def d3q7_state(torch, flb):
    """rho = 5 + sqrt(5) z on the device (torch generator, seed 0), f = w rho."""
    w, _ = flb.constants(3)
    g = torch.Generator(device="cuda").manual_seed(0)
    rho = 5.0 + np.sqrt(5.0) * torch.randn((512, 512, 512), generator=g, device="cuda", dtype=torch.float32)
    wt = torch.tensor(w, dtype=torch.float32, device="cuda").reshape(-1, 1, 1, 1)
    f0 = (wt * rho[None]).contiguous()
    del rho
    return f0


def leg_d3q7(torch, flb, tune, args, check=True):
    """D3Q7 512^3 FP32, omega = 1.2, rho = 5 + sqrt(5) z: the tuned kernel
    timed over max(K, 100) steps after the warmup, its rooflines, and its
    error against the oracle (the seeded state stepped 4 steps in the same
    launch configuration, 2000 sampled sites)."""
    dims = (512, 512, 512)
    N = 512 ** 3
    cfg = tune.best_config(3, 4, dims)
    f0 = d3q7_state(torch, flb)
    L = flb.Lattice(3, dims, precision=4, omega=1.2, seed=0, **cfg)
    se = args.sample_every
    L.set_populations(f0, step=(-args.warmup) % se if se else 0)
    if se:  # S(k) of the 768 axis modes and the lattice sums every se steps
        L.set_sampling(se, [(k, 0, 0) for k in range(1, 257)] + [(0, k, 0) for k in range(1, 257)]
                       + [(0, 0, k) for k in range(1, 257)])
        L.set_moment_sampling(se)
    L.step(args.warmup)
    steps = max(args.steps, 100)
    spl = steps_per_launch(cfg)
    steps -= steps % spl
    ms, kern = time_steps(torch, L, steps, se, spl)
    r, flat = roofline(kernel_name(cfg, d=3), kern * 1e3, 2 * 7 * 4 * N, spl, N)
    m = L.moments()
    out = {"workload": f"D3Q7 512^3 fp32 rho=5+sqrt(5)z, omega=1.2, S(k) of 768 axis modes and the lattice sums "
                       f"every {se} steps", "kernel": cfg, "steps": steps,
           "ms_per_step": round(ms, 4), "mlups": round(N / (ms * 1e-3) / 1e6, 1),
           "effective_gbs": flat["effective_gbs"], "hbm_frac_measured": flat["hbm_frac_measured"],
           "valu_frac": flat["valu_frac"], "roofline": r,
           "mass_drift_rel": (m["mass"] - m["mass0"]) / m["mass0"]}
    if check:
        log("D3Q7 oracle check")
        L.set_sampling(0)
        L.set_moment_sampling(0)
        L.set_populations(f0)
        L.step(4)
        out["oracle"] = sampled_error(L.get_populations(), f0.cpu().numpy(), 3, 1.2, 4, 5.0)
    L.close()
    del f0
    return out


def ensemble_members(torch, flb, inputs, keep=()):
    """The ensemble's lattices with seeded Poisson initial counts (on the
    device); host copies of the initial states of the members listed in keep."""
    g = torch.Generator(device="cuda").manual_seed(0)
    lats, kept = [], {}
    for i, r in enumerate(inputs.ensemble(1024, 256, seed=0)):
        w, _ = flb.constants(r["d"])
        L = flb.Lattice(r["d"], r["dims"], precision=4, omega=r["omega"], seed=r["seed"])
        shape = (len(w),) + tuple(reversed(r["dims"]))
        lam = torch.tensor(w * r["rho"], dtype=torch.float32, device="cuda").reshape((-1,) + (1,) * r["d"])
        f = torch.poisson(lam.expand(shape).contiguous(), generator=g)
        L.set_populations(f)
        if i in keep:
            kept[i] = f.cpu().numpy()
        lats.append(L)
    return lats, kept


def _check_members(flb, B, lats, reps, kept, steps):
    """Put the kept members back to their initial states, run the whole
    batch `steps` steps, and compare each kept member with the oracle's run
    of the same lattice: per member the max error, and the max over sites
    whose light cone saw no collision with |rho| < NEAR_ZERO[4].  The gate
    is the members at mean density >= 5; below a few particles per site FP32
    and FP64 trajectories part where the amplitude sqrt(max(rho, 0))
    magnifies rounding, and those members are reported apart."""
    import oracle
    for i in kept:
        B.retire(lats[i])
        lats[i].set_populations(kept[i], step=0)
        B.admit(lats[i])
    B.step(steps)
    B.sync()
    rows = []
    for i, f0 in kept.items():
        r = reps[i]
        B.retire(lats[i])
        g = lats[i].get_populations().astype(np.float64)
        B.admit(lats[i])
        lat = oracle.make_lattice(r["d"])
        p = oracle.Params(d=r["d"], omega_j=r["omega"], seed=r["seed"])
        ref, minrho = oracle.run_box(f0.astype(np.float64), lat, p, 0, steps, [0] * r["d"], r["dims"],
                                     horizon=min(steps, HORIZON))
        floor = (r["rho"] * lat.w).reshape((-1,) + (1,) * r["d"])
        err = np.abs(g - ref) / np.maximum(np.abs(ref), floor)
        ok = np.broadcast_to(minrho > NEAR_ZERO[4], err.shape)
        rows.append({"d": r["d"], "dims": list(r["dims"]), "rho": round(r["rho"], 3), "max_err": float(err.max()),
                     "max_err_well_conditioned": float(err[ok].max()) if ok.any() else None,
                     "sites_near_rho0": int((minrho <= NEAR_ZERO[4]).sum())})
    hi = [row["max_err"] for row in rows if row["rho"] >= 5.0]
    # members below rho 5 whose every site saw a near-zero collision have no
    # well-conditioned sites and contribute nothing here
    lo = [row["max_err_well_conditioned"] for row in rows
          if row["rho"] < 5.0 and row["max_err_well_conditioned"] is not None]
    return {"steps": steps, "members": rows, "max_err_rho_ge_5": max(hi) if hi else None,
            "max_err_rho_lt_5_well_conditioned": max(lo) if lo else None}


def leg_ensemble(torch, flb, inputs, tune, args, check=True):
    """1024 D1Q3 (L ~ U{64..4096}) + 256 D2Q5 (sides ~ U{128..1024}), FP32,
    per-replica seed / omega / density, Poisson initial counts, in one batch
    with the tuned options: max(K, 256) steps timed after max(W, 32) warmup
    steps; whole-step HBM and VALU fractions from the counted bytes and
    VALU cycles of every kernel of a step; and the oracle error of nine
    members (D1Q3 in LDS, D2Q5 in two-step passes) run again from their
    initial states inside the full batch."""
    reps = inputs.ensemble(1024, 256, seed=0)

    def smallest(d, dense, k):
        ids = [i for i, r in enumerate(reps) if r["d"] == d and (r["rho"] >= 5.0) == dense]
        return sorted(ids, key=lambda i: (np.prod(reps[i]["dims"]), i))[:k]
    # the gate: three D1Q3 (LDS) and three D2Q5 (two-step passes) members at
    # mean density >= 5, and the largest D1Q3; one low-density member of each
    # model reported apart
    big = max((i for i, r in enumerate(reps) if r["d"] == 1 and r["rho"] >= 5.0), key=lambda i: reps[i]["dims"][0])
    keep = tuple(smallest(1, True, 3) + [big] + smallest(2, True, 3) + smallest(1, False, 1) +
                 smallest(2, False, 1)) if check else ()
    bcfg = tune.batch_config()
    B = flb.Batch(**bcfg)
    lats, kept = ensemble_members(torch, flb, inputs, keep)
    log(f"ensemble of {len(lats)} lattices created")
    sites = 0
    for L in lats:
        B.admit(L)
        sites += L.nsite
    B.step(max(args.warmup, 32))
    B.sync()
    steps = max(args.steps, 256)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.step(steps)
    B.sync()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    bytes_step = sum(2 * L.Q * 4 * L.nsite for L in lats)
    n2 = sum(L.nsite for L in lats if L.d == 2)
    # counted bytes and VALU cycles of one step: per chunk of c steps the
    # LDS kernel runs once, the two-step kernel c/2 times, the advance once
    c = bcfg["chunk"]
    per_step = {"flb::k_batch_two<float, %d, 1>" % bcfg["width"]: 0.5, "flb::k_batch_lds_d1<float, 16, 1>": 1.0 / c,
                "flb::k_batch_advance<float>": 1.0 / c}
    tb = va = 0.0
    have = True
    for k, f in per_step.items():
        cnt = counters(k)
        if "traffic_bytes_per_launch" not in cnt or "valu_active_per_launch" not in cnt:
            have = have and k == "flb::k_batch_advance<float>"
            continue
        tb += f * cnt["traffic_bytes_per_launch"]
        va += f * cnt["valu_active_per_launch"]
    t = ms * 1e-3
    out = {"workload": "1024 D1Q3 L~U[64,4096] + 256 D2Q5 sides~U[128,1024], fp32, per-replica seed/omega/rho",
           "batch_options": bcfg, "replicas": len(lats), "sites": sites, "sites_d2q5": n2, "steps": steps,
           "ms_per_step": round(ms, 4), "mlups": round(sites / t / 1e6, 1),
           "effective_gbs": round(bytes_step / t / 1e9, 1),
           "hbm_frac_measured": round(tb / t / 1e9 / PEAK_HBM_GBS, 4) if have else None,
           "valu_frac": round(va / t / 1e9 / PEAK_VALU_G, 4) if have else None}
    if check:
        log("ensemble oracle check")
        out["oracle"] = _check_members(flb, B, lats, reps, kept, 2 * c + 1)
    for L in lats:
        B.retire(L)
        L.close()
    B.close()
    return out


def leg_served(torch, flb, args, n=16, budget_gib=4.0):
    """The served stream's first n requests (Poisson arrivals at 200/s,
    D1Q3/D2Q5/D3Q7, sites log-U[1e3, 1e8], steps log-U[1e2, 1e5], FP32,
    seed 0), served with an HBM budget of budget_gib under two storage
    policies: two buffers for every request, and the adaptive one (one
    buffer for D1Q3, two for D2Q5 and D3Q7 unless only the single-buffer
    footprint fits the free budget).  Per policy: makespan, throughput,
    p50/p99 latency and the requests resident at once."""
    from paper_1606_07801_amd import serve
    out = {"workload": f"served: first {n} requests of the Poisson(200/s) stream, seed 0, D1Q3/D2Q5/D3Q7, "
                       f"sites log-U[1e3,1e8], steps log-U[1e2,1e5], fp32, HBM budget {budget_gib} GiB"}
    for pol in ("two", "auto"):
        reqs = serve.make_requests(n, 200.0, seed=0)
        S = serve.Server(budget_bytes=int(budget_gib * 2 ** 30), layout=pol)
        mk = S.run(reqs)
        out[pol] = serve.summary(S, mk)
        S.close()
    return out


def _timed(torch, fn, steps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn(steps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def bench_d1q3(torch, flb, inputs, tune, args):
    """D1Q3, FP64, L = 256, 10^4 steps, Poisson counts at rho = 10, with the
    lattice sums and S(k) of all 255 nonzero modes taken every step; also
    timed without sampling."""
    dims = (256,)
    w, _ = flb.constants(1)
    cfg = tune.best_config(1, 8, dims)
    f0 = inputs.poisson_counts(dims, 10.0 * w, seed=0)
    steps = 10_000
    L = flb.Lattice(1, dims, precision=8, omega=1.0, seed=0, **cfg)
    L.set_populations(f0)
    L.step(args.warmup)
    ms_plain = _timed(torch, L.step, steps)
    L.close()
    L = flb.Lattice(1, dims, precision=8, omega=1.0, seed=0, **cfg)
    L.set_populations(f0)
    ks = [[k] for k in range(1, 256)]
    L.set_moment_sampling(1)
    L.set_sampling(1, ks)
    ms = _timed(torch, L.step, steps)
    sums, n = L.sampled_moments()
    S = L.structure_factor(mode="read")[:255]
    m = L.moments()
    L.close()
    return {"workload": "D1Q3 256 fp64 rho=10 Poisson, omega=1, 10^4 steps, lattice sums and S(k) of all 255 "
                        "k != 0 every step", "kernel": cfg, "ms_per_step": round(ms, 6),
            "mlups": round(256 / ms / 1e3, 2), "ms_per_step_unsampled": round(ms_plain, 6),
            "mlups_unsampled": round(256 / ms_plain / 1e3, 2), "samples": n,
            "mass_drift": m["mass"] - m["mass0"], "mean_mass": sums["mass"] / n,
            "sk_mean_over_rho": round(float(S.mean() / (m["mass"] / 256)), 4),
            "ms_per_step_one_launch_per_step": round(_d1q3_launch_per_step(torch, flb, f0, ks), 6),
            **({} if args.no_cpu_baseline else {"cpu_baseline": cpu_baseline_d1q3(flb, f0, cfg)})}


def _scaled_err(g, ref, rho, w):
    """max |g - ref| / max(|ref|, rho_mean w_i): the tests' tolerance scale."""
    d = ref.ndim - 1
    floor = rho * np.asarray(w).reshape((-1,) + (1,) * d)
    return float((np.abs(np.asarray(g, dtype=np.float64) - ref) / np.maximum(np.abs(ref), floor)).max())


def cpu_baseline_d1q3(flb, f0, cfg):
    """The oracle on the whole D1Q3 workload (256 sites, 10^4 steps, one
    core), and the GPU's final state against it (all populations)."""
    import oracle
    p = oracle.Params(d=1, omega_j=1.0, seed=0)
    t0 = time.perf_counter()
    ref = oracle.run(np.asarray(f0, dtype=np.float64), p, 10_000)
    dt = time.perf_counter() - t0
    L = flb.Lattice(1, (256,), precision=8, omega=1.0, seed=0, **cfg)
    L.set_populations(f0)
    L.step(10_000)
    g = L.get_populations()
    L.close()
    return {"value": round(256 * 10_000 / dt / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"the whole workload: 256 sites x 10^4 steps ({dt:.1f} s)",
            "gpu_fp64_max_err_vs_oracle": _scaled_err(g, ref, 10.0, oracle.make_lattice(1).w)}


def _d1q3_launch_per_step(torch, flb, f0, ks):
    """The same sampled run on the HBM kernels (one launch per step and per
    statistic), for comparison."""
    L = flb.Lattice(1, (256,), precision=8, omega=1.0, seed=0, kernel="flat", tile_rows=1)
    L.set_populations(f0)
    L.set_moment_sampling(1)
    L.set_sampling(1, ks)
    ms = _timed(torch, L.step, 2000)
    L.close()
    return ms


def bench_d3q7(torch, flb, inputs, tune, args):
    """D3Q7, FP32 populations, 512^3, rho = 5 + sqrt(5) z, omega = 1.2, 500
    steps (the leg of the default line with 500 timed steps), plus the
    oracle's rate on one full step of a 512 x 512 x 128 slab."""
    args.steps = 500
    out = leg_d3q7(torch, flb, tune, args, check=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_d3q7(inputs)
    return out


def cpu_baseline_d3q7(inputs):
    """The oracle's rate on one core: one full step of a 512 x 512 x 128
    periodic slab of the same kind of seeded Gaussian state (the per-site
    work of the 512^3 step)."""
    import contextlib

    import oracle
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    lat = oracle.make_lattice(3)
    p = oracle.Params(d=3, omega_j=1.2, seed=0)
    slab = (512, 512, 128)
    fs = inputs.outer(lat.w, inputs.gaussian_field(slab, 5.0, np.sqrt(5.0), seed=2)).astype(np.float64)
    with threadpool_limits(limits=1) if threadpool_limits else contextlib.nullcontext():
        t0 = time.perf_counter()
        oracle.step(fs, lat, p, 0)
        dt = time.perf_counter() - t0
    n = slab[0] * slab[1] * slab[2]
    return {"value": round(n / dt / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"one step of a 512x512x128 periodic slab ({dt:.1f} s)"}


def bench_batched(torch, flb, inputs, tune, args):
    """The ensemble leg of the default line with 2000 timed steps, plus the
    oracle's rate on a sample of the ensemble."""
    args.steps = 2000
    out = leg_ensemble(torch, flb, inputs, tune, args, check=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(flb, inputs, tune.batch_config())
    return out


def cpu_baseline_batched(flb, inputs, bcfg, steps=100):
    """The oracle on a bounded sample of the ensemble: the first two D1Q3 and
    the first two D2Q5 replicas (seeded Poisson counts), `steps` steps each,
    timed on one core; the same replicas run as a batch with the benchmark's
    options, compared population by population (the tests' scale:
    max(|f|, rho_mean w_i)).  Below a few particles per site FP32 rounding
    reaches the noise amplitude sqrt(max(rho, 0)) as sqrt(rounding), so FP32
    and FP64 trajectories of such replicas part over many steps; the error
    of the replicas at mean density >= 5 is reported apart, and the same
    replicas are also run as an FP64 batch."""
    import oracle
    reps = inputs.ensemble(1024, 256, seed=0)
    pick = [r for r in reps if r["d"] == 1][:2] + [r for r in reps if r["d"] == 2][:2]
    B = flb.Batch(**bcfg)
    runs, dt, work = [], 0.0, 0
    for r in pick:
        lat = oracle.make_lattice(r["d"])
        f0 = inputs.poisson_counts(r["dims"], r["rho"] * lat.w, seed=r["seed"]).astype(np.float32)
        L = flb.Lattice(r["d"], r["dims"], precision=4, omega=r["omega"], seed=r["seed"])
        L.set_populations(f0)
        B.admit(L)
        runs.append((r, lat, f0, L))
    B.step(steps)
    B.sync()
    per, refs = [], []
    for r, lat, f0, L in runs:
        B.retire(L)
        g = L.get_populations()
        L.close()
        t0 = time.perf_counter()
        ref = oracle.run(f0.astype(np.float64), oracle.Params(d=r["d"], omega_j=r["omega"], seed=r["seed"]), steps)
        dt += time.perf_counter() - t0
        refs.append(ref)
        work += int(np.prod(r["dims"])) * steps
        per.append({"d": r["d"], "dims": list(r["dims"]), "rho": round(r["rho"], 3),
                    "max_err": _scaled_err(g, ref, r["rho"], lat.w)})
    B.close()
    B = flb.Batch(**bcfg)
    lats = []
    for r, lat, f0, _ in runs:
        L = flb.Lattice(r["d"], r["dims"], precision=8, omega=r["omega"], seed=r["seed"])
        L.set_populations(f0.astype(np.float64))
        B.admit(L)
        lats.append(L)
    B.step(steps)
    B.sync()
    for (r, lat, _, _), L, ref, row in zip(runs, lats, refs, per):
        B.retire(L)
        row["max_err_fp64"] = _scaled_err(L.get_populations(), ref, r["rho"], lat.w)
        L.close()
    B.close()
    hi = [row["max_err"] for row in per if row["rho"] >= 5.0]
    return {"value": round(work / dt / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"2 D1Q3 + 2 D2Q5 replicas x {steps} steps ({dt:.1f} s)",
            "gpu_fp32_max_err_rho_ge_5": max(hi) if hi else None,
            "gpu_fp32_max_err_all": max(row["max_err"] for row in per),
            "gpu_fp64_max_err_all": max(row["max_err_fp64"] for row in per), "per_replica": per}


def bench_served(torch, flb, inputs, tune, args):
    """The configured stream (Poisson arrivals at 200 requests/s, about 250
    times what one GPU serves, so latency is mostly queueing), then the same
    requests arriving at 0.5 and 0.9 of the capacity that run measured
    (site-updates per second over the mean work per request)."""
    from paper_1606_07801_amd import serve

    def run(rate):
        reqs = serve.make_requests(args.requests, rate, seed=0)
        S = serve.Server()
        mk = S.run(reqs, progress=30.0)
        res = serve.summary(S, mk)
        res["rate_per_s"] = round(rate, 4)
        S.close()
        return res, reqs

    out, reqs = run(200.0)
    cap = out["mlups"] * 1e6                                   # site-updates per second
    mean_work = float(np.mean([r.sites * r.steps for r in reqs]))
    out["workload"] = ("served: Poisson arrivals 200/s, D1Q3/D2Q5/D3Q7, sites log-U[1e3,1e8], "
                       "steps log-U[1e2,1e5], fp32")
    out["capacity_requests_per_s"] = round(cap / mean_work, 4)
    for frac in (0.5, 0.9):
        res, _ = run(frac * cap / mean_work)
        out[f"at_{frac}_of_capacity"] = res
    # the same stream with a constrained budget under both storage policies
    for pol in ("two", "auto"):
        reqs = serve.make_requests(args.requests, 200.0, seed=0)
        S = serve.Server(budget_bytes=8 << 30, layout=pol)
        mk = S.run(reqs, progress=30.0)
        out[f"budget_8gib_{pol}"] = serve.summary(S, mk)
        S.close()
    if not args.no_cpu_baseline:
        out["oracle_check"] = served_oracle_check(serve, reqs)
    return out


def served_oracle_check(serve, reqs, count=3, max_work=2e7, min_rho=5.0):
    """The `count` cheapest requests of the stream with mean density at least
    `min_rho` (away from the clamp at zero, where FP32 and FP64 trajectories
    may part) and at most `max_work` site-updates, served together with
    their final states kept, against the oracle's FP64 run of the same
    request from the same initial state."""
    import oracle
    pick = sorted((r for r in reqs if r.rho >= min_rho and r.sites * r.steps <= max_work),
                  key=lambda r: r.sites * r.steps)[:count]
    if not pick:
        return None
    again = [serve.Request(i, 0.0, r.d, r.dims, r.steps, r.omega, r.rho, r.seed, keep_state=True)
             for i, r in enumerate(pick)]
    S = serve.Server()
    S.run(again)
    S.close()
    rows, worst = [], 0.0
    for r in again:
        lat = oracle.make_lattice(r.d)
        f0 = np.broadcast_to((np.float32(r.rho) * lat.w.astype(np.float32)).reshape((-1,) + (1,) * r.d),
                             (lat.Q,) + tuple(reversed(r.dims))).astype(np.float64)
        fo = oracle.run(f0, oracle.Params(d=r.d, omega_j=r.omega, seed=r.seed), r.steps)
        g = r.result["state"].astype(np.float64)
        err = _scaled_err(g, fo, r.rho, lat.w)
        worst = max(worst, err)
        rows.append({"d": r.d, "dims": list(r.dims), "steps": r.steps, "rho": round(r.rho, 3),
                     "max_err": err})
    return {"requests": rows, "gpu_fp32_max_err_vs_oracle": worst}


OTHER = {"d1q3": bench_d1q3, "d3q7": bench_d3q7, "batched": bench_batched, "served": bench_served}


if __name__ == "__main__":
    main()
