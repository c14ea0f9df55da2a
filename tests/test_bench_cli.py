"""bench.py on the host: the argument parser, the kernel names it reports,
the counter-summary reader, the roofline object, and the refusal of
multi-GPU runs."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_parse_defaults(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert a.gpus == 1 and a.steps > 0 and a.warmup >= 0 and a.workload == "lattice"


def test_kernel_names():
    assert bench.kernel_name({"kernel": "two", "tile_rows": 8, "nt_store": 1}) == "flb::k_step2_d2<float, 8, true, false, 1>"
    assert bench.kernel_name({"kernel": "flat", "tile_rows": 2, "nt_store": 1}) == "flb::k_step_flat<2, float, 2, true, 1>"
    assert bench.kernel_name({"kernel": "flat", "tile_rows": 1, "nt_store": 1}, d=3) == "flb::k_step_flat<3, float, 1, true, 1>"
    assert bench.kernel_name({"kernel": "plain"}, prec="double") == "flb::k_step_plain<2, double>"
    assert bench.steps_per_launch({"kernel": "two"}) == 2 and bench.steps_per_launch({"kernel": "flat"}) == 1


def test_traffic_reader_unknown_kernel_is_none():
    assert bench.measured_traffic("no such kernel") is None
    assert bench.counters("no such kernel") == {}


def test_multi_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def _summary(tmp_path, src, k):
    p = tmp_path / "summary.md"
    p.write_text(f"# t\n\n```\nkernel_source_sha256_16: {src}\nkernel: {k}\n"
                 f"traffic_bytes_per_launch: 1000000\nvalu_wave_insts_per_launch: 614400\n"
                 f"valu_active_per_launch: 921600\nvalu_busy: 0.9\nkernel: other\n"
                 f"traffic_bytes_per_launch: 5\n```\n")
    return str(p)


def test_counter_summary_reader_and_roofline(tmp_path, monkeypatch):
    k = "flb::k_step2_d2<float, 8, true, false, 1>"
    path = _summary(tmp_path, bench.source_hash(), k)
    monkeypatch.setattr(bench, "COUNTER_FILES", [path])
    c = bench.counters(k)
    assert c["traffic_bytes_per_launch"] == 1e6 and c["valu_active_per_launch"] == 921600
    assert bench.counters("other") == {"traffic_bytes_per_launch": 5.0}
    # 1 ms launch: 1 GB/s counted traffic, 0.9216 G quad-cycles/s of VALU
    r, flat = bench.roofline(k, 1000.0, 4_000_000, 2, 1000)
    assert r["bound"] == "alu" and r["unit"] == "G VALU quad-cycles/s"
    assert abs(r["frac"] - 0.9216 / 614.4) < 1e-6 and r["frac"] <= 1
    assert r["hbm"]["bytes"] == "counted" and abs(r["hbm"]["achieved"] - 1.0) < 1e-9
    assert abs(r["alu"]["issue_frac"] - 0.6144 / 614.4) < 1e-6
    assert flat["effective_gbs"] == 8.0 and flat["kernel_mlups"] == 2.0
    # summaries taken on other sources are ignored: the HBM roofline on the
    # algorithmic bytes of the launch
    monkeypatch.setattr(bench, "COUNTER_FILES", [_summary(tmp_path, "0" * 16, k)])
    assert bench.counters(k) == {} and bench.measured_traffic(k) is None
    r, flat = bench.roofline(k, 1000.0, 4_000_000, 2, 1000)
    assert r["bound"] == "hbm" and r["traffic"] is None and r["hbm"]["bytes"] == "algorithmic"
    assert flat["hbm_frac_measured"] is None and flat["valu_frac"] is None


def test_sk_flatness_statistic():
    # exact stationary values give zero z; the sine mode is excluded
    import numpy as np
    kv = [(k, 0) for k in range(1, 9)] + [(0, k) for k in range(1, 9)]
    S = np.full(len(kv), 10.0)
    S[0] = 500.0
    r = bench.sk_flatness(S, kv, 64, 10.0, [0, 10, 20], {(1, 0)})
    assert r["modes"] == 15 and r["mean_ratio"] == 1.0 and r["max_abs_z"] == 0.0
