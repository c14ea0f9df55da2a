"""Benchmark of the fluctuating lattice Boltzmann step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (one "step" = one pass of the hot path over the lattice): a D2Q5
lattice of 4096 x 4096 sites, float32 populations, mean density 10 with a
sine mode of relative amplitude 0.1, omega = 1, local Gaussian noise, seed 0;
every step runs the fused stream-collide kernel, and every `--sample-every`
steps (default 10) the sampled variant of the step also accumulates the FP64
density marginals, from which the structure factor of 1024 axis modes is
accumulated on the device; the FP64 lattice sums are taken at the end.
Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
PEAK_VALU_GINST = 256 * 2.4  # G wave64 VALU instructions/s: 256 CUs, one per CU per clock at 2.4 GHz
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "step_d2q5_4096_fp32_traffic.md")


def measured_counter(kernel, key="traffic_bytes_per_launch"):
    """A per-launch counter figure of `kernel` from the committed counter
    summary (key "traffic_bytes_per_launch": HBM bytes; key
    "valu_wave_insts_per_launch": VALU instructions issued, wave-level), or
    None if the step kernels' sources changed since the counters were taken
    or the summary has no such entry.  The summary lists blocks of
    "kernel: <name>" followed by "<key>: <n>" lines."""
    import hashlib
    try:
        entries, cur, src = {}, None, None
        for line in open(TRAFFIC_PROFILE):
            if ":" not in line or line.startswith(("#", "|", " ", "`")):
                continue
            k, v = (x.strip() for x in line.split(":", 1))
            if k == "kernel_source_sha256_16":
                src = v
            elif k == "kernel":
                cur = v
            elif k == key and cur:
                entries[cur] = int(float(v))
        h = hashlib.sha256()
        for f in ("flb_device.hpp", "flb_kernels.hpp"):
            with open(os.path.join(ROOT, "paper_1606_07801_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest()[:16] != src:
            return None
        return entries.get(kernel)
    except (OSError, ValueError):
        return None


def measured_traffic(kernel):
    return measured_counter(kernel, "traffic_bytes_per_launch")


def valu_issue(kernel, us):
    """VALU issue rate of a launch of `kernel` lasting `us`: the counted
    wave-level VALU instructions per launch over the time, against the
    chip's issue peak (one wave64 instruction per CU per clock: a 16-lane
    SIMD takes four clocks per instruction and a CU has four SIMDs)."""
    n = measured_counter(kernel, "valu_wave_insts_per_launch")
    if not n:
        return None
    rate = n / (us * 1e-6) / 1e9
    return {"wave_insts_per_launch": n, "achieved": round(rate, 1), "peak": PEAK_VALU_GINST,
            "unit": "G wave-instructions/s", "frac": round(rate / PEAK_VALU_GINST, 4)}




def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--sample-every", type=int, default=10)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--requests", type=int, default=48, help="served workload: number of requests")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--workload", default="lattice", choices=["lattice", "d1q3", "d3q7", "batched", "served"],
                    help="lattice: the D2Q5 4096^2 line (default); the others print their own line")
    return ap.parse_args()


def kernel_name(cfg):
    """Name of the step kernel a launch configuration selects (as profiled)
    for the benchmark's local Gaussian noise (the two-step kernel's instance
    with that noise plan fixed at compile time, plan 1)."""
    nt = "true" if cfg.get("nt_store") else "false"
    if cfg.get("kernel") == "two":
        ty = cfg.get("tile_rows") or 8
        return f"flb::k_step2_d2<float, {2 if ty <= 2 else ty}, {nt}, false, 1>"
    if cfg.get("kernel") == "flat":
        return f"flb::k_step_flat<2, float, {cfg.get('tile_rows') or 2}, {nt}>"
    if cfg.get("kernel") == "plain":
        return "flb::k_step_plain<2, float>"
    return f"flb::k_step_rows<2, float, {cfg.get('tile_rows') or 4}, {nt}>"


def workload_state(flb, inputs, n, precision):
    w, _ = flb.constants(2)
    rho = inputs.sine_field((n, n), 10.0, 0.1)
    return inputs.outer(w, rho).astype(np.float32 if precision == 4 else np.float64)


def steps_per_launch(cfg):
    """Steps one launch of the dominant step kernel advances."""
    return 2 if cfg.get("kernel") == "two" else 1


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
    return (t1 - t0) * 1e3 / steps, total / launches


def depth1_reference(torch, flb, f0, dims):
    """The one-step flat kernel on the same lattice (each step reads and
    writes every population once): its duration and HBM roofline fraction,
    the reference for the two-step pass."""
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
    L.close()
    us = e0.elapsed_time(e1) * 1e3 / 100
    name = kernel_name(cfg)
    nbytes = 2 * 5 * 4 * dims[0] * dims[1]
    gbs = nbytes / (us * 1e-6) / 1e9
    return {"kernel": name, "kernel_us": round(us, 2), "achieved": round(gbs, 1),
            "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": measured_traffic(name),
            "valu": valu_issue(name, us)}


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
    f0 = workload_state(flb, inputs, n, 4)
    L = flb.Lattice(2, dims, precision=4, omega=1.0, seed=0, noise="local", **cfg)
    L.set_populations(f0)
    kvecs = [(k, 0) for k in range(1, 513)] + [(0, k) for k in range(1, 513)]
    if args.sample_every:
        L.set_sampling(args.sample_every, kvecs)

    # warmup, then the timed region (all hot-path rows: step + sampled stats)
    L.step(args.warmup)
    spl = steps_per_launch(cfg)
    ms_step, kern_ms = time_steps(torch, L, args.steps, args.sample_every, spl)
    m = L.moments()
    S = L.structure_factor(None, mode="read")[:len(kvecs)] if args.sample_every else np.zeros(1)
    L.close()
    depth1 = depth1_reference(torch, flb, f0, dims)

    value = N / (ms_step * 1e-3) / 1e6  # MLUPS of the whole job
    # algorithmic: every step reads and writes every population once; a
    # launch of the two-step kernel advances two steps
    bytes_per_launch = spl * 2 * Q * 4 * N
    achieved = bytes_per_launch / (kern_ms * 1e-3) / 1e9
    traffic = measured_traffic(kernel_name(cfg))

    out = {
        "metric": "MLUPS", "value": round(value, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"D2Q5 {n}x{n} periodic, fp32 populations, rho=10 sine mode 0.1, "
                        f"omega=1.0, local Gaussian noise (Philox), S(k) of 1024 axis modes "
                        f"accumulated every {args.sample_every} steps, lattice sums at the end",
            "kernel": cfg, "sites": N,
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "kernel": kernel_name(cfg), "kernel_us": round(kern_ms * 1e3, 2),
            "bytes_per_launch": bytes_per_launch, "steps_per_launch": spl,
            "measured_hbm_gbs": round(traffic / (kern_ms * 1e-3) / 1e9, 1) if traffic else None,
            "valu": valu_issue(kernel_name(cfg), kern_ms * 1e3),
        },
        "step_kernel_mlups": round(spl * N / (kern_ms * 1e-3) / 1e6, 1),
        "depth1": depth1,
        "mass_drift_rel": abs(m["mass"] - m["mass0"]) / m["mass0"],
        "sk_median_over_rho": float(np.median(S) / m["rho_eq"]),
    }

    if not args.no_fp64:
        # comparator: the plain FP64 single-lattice path on the same GPU
        f64 = workload_state(flb, inputs, n, 8)
        P = flb.Lattice(2, dims, precision=8, omega=1.0, seed=0, kernel="plain")
        P.set_populations(f64)
        P.step(10)
        k64 = max(args.steps // 4, 20)
        ms64, kern64 = time_steps(torch, P, k64, 0)
        P.close()
        out["fp64_plain"] = {"mlups": round(N / (ms64 * 1e-3) / 1e6, 1), "ms_per_step": round(ms64, 4),
                             "hbm_gbs": round(2 * Q * 8 * N / (kern64 * 1e-3) / 1e9, 1)}
        # the tuned FP64 path (same state, same steps, no sampling)
        cfg64 = tune.best_config(2, 8, dims)
        P = flb.Lattice(2, dims, precision=8, omega=1.0, seed=0, **cfg64)
        P.set_populations(f64)
        P.step(10)
        spl64 = steps_per_launch(cfg64)
        ms64, kern64 = time_steps(torch, P, k64, 0, spl64)
        P.close()
        out["fp64_tuned"] = {"kernel": cfg64, "mlups": round(N / (ms64 * 1e-3) / 1e6, 1),
                             "ms_per_step": round(ms64, 4),
                             "effective_gbs": round(spl64 * 2 * Q * 8 * N / (kern64 * 1e-3) / 1e9, 1)}

    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 10
        out["copy_probe"] = {"bytes_each_way": nb, "gbs_read_plus_write": round(2 * nb / dt / 1e9, 1)}
        del src, dst

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(flb, inputs, n, f0)

    print(json.dumps(out), flush=True)


def cpu_baseline(flb, inputs, n, f0):
    """The FP64 oracle (single-threaded numpy) on a bounded sample of the
    same workload: 4 steps of the full lattice from the seeded state.  The
    GPU path's result from the same state is compared with it, every
    population; sites within reach of a collision with |rho| < 1e-3 (where
    the noise amplitude sqrt(max(rho, 0)) is not Lipschitz) during those
    steps are counted apart."""
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
        ref = f0.astype(np.float64)
        for t in range(nsteps):
            near.append(np.abs(ref.sum(axis=0)) < 1e-3)  # collisions of step t near rho = 0
            t0 = time.perf_counter()
            ref = oracle.step(ref, lat, p, t)
            dt += time.perf_counter() - t0
    L = flb.Lattice(2, (n, n), precision=4, omega=1.0, seed=0, noise="local")
    L.set_populations(f0)
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
            "gpu_fp32_max_err_vs_oracle": float(err.max()),
            "gpu_fp32_max_err_well_conditioned": float(err[~flag].max()),
            "n_pops_near_rho0_reach": int(flag.sum())}


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
    """D3Q7, FP32 populations, 512^3, rho = 5 + sqrt(5) z, omega = 1.2, 500 steps."""
    dims = (512, 512, 512)
    N = 512 ** 3
    w, _ = flb.constants(3)
    cfg = tune.best_config(3, 4, dims)
    L = flb.Lattice(3, dims, precision=4, omega=1.2, seed=0, **cfg)
    g = torch.Generator(device="cuda").manual_seed(0)
    rho = 5.0 + np.sqrt(5.0) * torch.randn((512, 512, 512), generator=g, device="cuda", dtype=torch.float32)
    wt = torch.tensor(w, dtype=torch.float32, device="cuda").reshape(-1, 1, 1, 1)
    L.set_populations((wt * rho[None]).contiguous())
    del rho
    L.step(20)
    steps = 500
    ms = _timed(torch, L.step, steps)
    m = L.moments()
    L.close()
    gbs = 2 * 7 * 4 * N / (ms * 1e-3) / 1e9
    out = {"workload": "D3Q7 512^3 fp32 rho=5+sqrt(5)z, omega=1.2, 500 steps", "kernel": cfg,
           "ms_per_step": round(ms, 4), "mlups": round(N / (ms * 1e-3) / 1e6, 1),
           "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4),
           "mass_drift_rel": (m["mass"] - m["mass0"]) / m["mass0"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_d3q7(flb, inputs, cfg)
    return out


def cpu_baseline_d3q7(flb, inputs, cfg, nsample=2000):
    """The oracle on a bounded sample of the D3Q7 workload, on one core: its
    rate from one full step of a 512 x 512 x 128 periodic slab of the same
    kind of seeded Gaussian state (the per-site work of the 512^3 step); its
    error against the GPU from one step of `nsample` sites of the seeded
    512^3 state (each site on its own 3 x 3 x 3 window), compared with the
    GPU's step of the whole lattice in the benchmark's launch configuration."""
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
    del fs
    dims = (512, 512, 512)
    rho = inputs.gaussian_field(dims, 5.0, np.sqrt(5.0), seed=0)
    f0 = inputs.outer(lat.w, rho).astype(np.float32)
    del rho
    coords = inputs.rng(1).integers(0, 512, size=(nsample, 3))
    ref = oracle.run_sites(f0, lat, p, 0, 1, coords)
    L = flb.Lattice(3, dims, precision=4, omega=1.2, seed=0, **cfg)
    L.set_populations(f0)
    L.step(1)
    g = L.get_populations()
    L.close()
    got = g[:, coords[:, 2], coords[:, 1], coords[:, 0]].astype(np.float64)
    floor = 5.0 * lat.w[:, None]
    err = float((np.abs(got - ref) / np.maximum(np.abs(ref), floor)).max())
    n = slab[0] * slab[1] * slab[2]
    return {"value": round(n / dt / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"one step of a 512x512x128 periodic slab ({dt:.1f} s); error at {nsample} sampled "
                      f"sites of one step of the 512^3 lattice",
            "gpu_fp32_max_err_vs_oracle": err}


def ensemble_members(torch, flb, inputs):
    """The ensemble's lattices with seeded Poisson initial counts (on the device)."""
    g = torch.Generator(device="cuda").manual_seed(0)
    lats = []
    for r in inputs.ensemble(1024, 256, seed=0):
        w, _ = flb.constants(r["d"])
        L = flb.Lattice(r["d"], r["dims"], precision=4, omega=r["omega"], seed=r["seed"])
        shape = (len(w),) + tuple(reversed(r["dims"]))
        lam = torch.tensor(w * r["rho"], dtype=torch.float32, device="cuda").reshape((-1,) + (1,) * r["d"])
        L.set_populations(torch.poisson(lam.expand(shape).contiguous(), generator=g))
        lats.append(L)
    return lats


def bench_batched(torch, flb, inputs, tune, args):
    """1024 D1Q3 (L ~ U{64..4096}) + 256 D2Q5 (sides ~ U{128..1024}), FP32,
    per-replica seed / omega / density, Poisson initial counts, 2000 steps."""
    bcfg = tune.batch_config()
    B = flb.Batch(**bcfg)
    lats = ensemble_members(torch, flb, inputs)
    sites = 0
    for L in lats:
        B.admit(L)
        sites += L.nsite
    B.step(32)
    steps = 2000
    ms = _timed(torch, lambda n: (B.step(n), B.sync()), steps)
    bytes_step = sum(2 * L.Q * 4 * L.nsite for L in lats)
    for L in lats:
        B.retire(L)
        L.close()
    B.close()
    out = {"workload": "batched: 1024 D1Q3 L~U[64,4096] + 256 D2Q5 sides~U[128,1024], fp32, 2000 steps",
           "batch_options": bcfg, "replicas": len(lats), "sites": sites, "ms_per_step": round(ms, 4),
           "mlups": round(sites / (ms * 1e-3) / 1e6, 1),
           "effective_gbs": round(bytes_step / (ms * 1e-3) / 1e9, 1)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(flb, inputs, bcfg)
    return out


def cpu_baseline_batched(flb, inputs, bcfg, steps=100):
    """The oracle on a bounded sample of the ensemble: the first two D1Q3 and
    the first two D2Q5 replicas (seeded Poisson counts), `steps` steps each,
    timed on one core; the same replicas run as a batch with the benchmark's
    options, compared population by population."""
    import oracle
    reps = inputs.ensemble(1024, 256, seed=0)
    pick = [r for r in reps if r["d"] == 1][:2] + [r for r in reps if r["d"] == 2][:2]
    B = flb.Batch(**bcfg)
    runs, dt, work, err = [], 0.0, 0, 0.0
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
        e = _scaled_err(g, ref, max(r["rho"], 1.0), lat.w)
        err = max(err, e)
        # below a few particles per site FP32 rounding reaches the noise
        # amplitude sqrt(max(rho, 0)) as sqrt(rounding), so the trajectories
        # separate over many steps; the error is reported with the density
        per.append({"d": r["d"], "dims": list(r["dims"]), "rho": round(r["rho"], 3), "max_err": e})
    B.close()
    # the same replicas with FP64 populations in a batch of their own: no
    # such separation, so the whole trajectory matches the oracle
    B = flb.Batch(**bcfg)
    lats = []
    for r, lat, f0, _ in runs:
        L = flb.Lattice(r["d"], r["dims"], precision=8, omega=r["omega"], seed=r["seed"])
        L.set_populations(f0.astype(np.float64))
        B.admit(L)
        lats.append(L)
    B.step(steps)
    B.sync()
    err64 = 0.0
    for (r, lat, _, _), L, ref, row in zip(runs, lats, refs, per):
        B.retire(L)
        e = _scaled_err(L.get_populations(), ref, max(r["rho"], 1.0), lat.w)
        L.close()
        row["max_err_fp64"] = e
        err64 = max(err64, e)
    B.close()
    return {"value": round(work / dt / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"2 D1Q3 + 2 D2Q5 replicas x {steps} steps ({dt:.1f} s)",
            "gpu_fp32_max_err_vs_oracle": err, "gpu_fp64_max_err_vs_oracle": err64, "per_replica": per}


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
        scale = np.maximum(np.abs(fo), (r.rho * lat.w).reshape((-1,) + (1,) * r.d))
        err = float(np.max(np.abs(g - fo) / scale))
        worst = max(worst, err)
        rows.append({"d": r.d, "dims": list(r.dims), "steps": r.steps, "rho": round(r.rho, 3),
                     "max_err": err})
    return {"requests": rows, "gpu_fp32_max_err_vs_oracle": worst}


OTHER = {"d1q3": bench_d1q3, "d3q7": bench_d3q7, "batched": bench_batched, "served": bench_served}


if __name__ == "__main__":
    main()
