"""bench.py on the host: the argument parser, the kernel names it reports,
the traffic-summary reader, and the refusal of multi-GPU runs."""

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
    assert bench.kernel_name({"kernel": "flat", "tile_rows": 2, "nt_store": 1}) == "flb::k_step_flat<2, float, 2, true>"
    assert bench.steps_per_launch({"kernel": "two"}) == 2 and bench.steps_per_launch({"kernel": "flat"}) == 1


def test_traffic_reader_unknown_kernel_is_none():
    assert bench.measured_traffic("no such kernel") is None


def test_multi_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_counter_summary_reader(tmp_path, monkeypatch):
    import hashlib
    h = hashlib.sha256()
    for f in ("flb_device.hpp", "flb_kernels.hpp"):
        with open(os.path.join(ROOT, "paper_1606_07801_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    k = "flb::k_step2_d2<float, 8, true, false, 1>"
    summary = tmp_path / "summary.md"
    summary.write_text(f"# t\n\n```\nkernel_source_sha256_16: {h.hexdigest()[:16]}\nkernel: {k}\n"
                       f"traffic_bytes_per_launch: 1000\nvalu_wave_insts_per_launch: 614400\n```\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(summary))
    assert bench.measured_traffic(k) == 1000
    v = bench.valu_issue(k, 1000.0)                 # 614,400 instructions in 1 ms
    assert v["achieved"] == 0.6 and v["frac"] == 0.001          # 0.6144 G/s of 614.4
    # a summary taken on other sources is ignored
    summary.write_text(summary.read_text().replace(h.hexdigest()[:16], "0" * 16))
    assert bench.measured_traffic(k) is None and bench.valu_issue(k, 1000.0) is None
