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
    assert bench.kernel_name({"kernel": "two", "tile_rows": 8, "nt_store": 1}) == "flb::k_step2_d2<float, 8, true, false>"
    assert bench.kernel_name({"kernel": "flat", "tile_rows": 2, "nt_store": 1}) == "flb::k_step_flat<2, float, 2, true>"
    assert bench.steps_per_launch({"kernel": "two"}) == 2 and bench.steps_per_launch({"kernel": "flat"}) == 1


def test_traffic_reader_unknown_kernel_is_none():
    assert bench.measured_traffic("no such kernel") is None


def test_multi_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
