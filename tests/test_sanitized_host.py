"""The library's host code under AddressSanitizer and UndefinedBehavior-
Sanitizer, on the CPU: the C client (compiled with the same clang
sanitizers, leak detection on) and the host-side ABI tests (a Python
process with the ASan runtime preloaded) against lib/libflb_san.so, built by
`python -m paper_1606_07801_amd.build --sanitize` (device code as usual,
sanitizers on the host side only).  Skipped when that build is absent or
older than the sources."""

import os
import subprocess
import sys

import pytest

from paper_1606_07801_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")

def _stale():
    """The sanitized build predates a source it is built from."""
    srcs = [os.path.join(build.CSRC, f) for f in os.listdir(build.CSRC)] + [os.path.join(ROOT, "include", "flb.h")]
    return os.path.getmtime(build.LIB_SAN) < max(os.path.getmtime(f) for f in srcs)


pytestmark = [
    pytest.mark.skipif(not os.path.exists(build.LIB_SAN) or build.sanitizer_runtime() is None
                       or not os.path.exists(CLANG),
                       reason="no sanitized build (python -m paper_1606_07801_amd.build --sanitize)"),
    pytest.mark.skipif(os.path.exists(build.LIB_SAN) and _stale(),
                       reason="the sanitized build is older than the sources; rebuild it with "
                              "python -m paper_1606_07801_amd.build --sanitize"),
]


def test_c_client_under_asan_ubsan(tmp_path):
    libdir = os.path.dirname(build.LIB_SAN)
    exe = str(tmp_path / "c_client_san")
    subprocess.run([CLANG, "-std=c99", "-Wall", "-Wextra", "-Werror", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_client.c"), "-o", exe, "-L", libdir, "-lflb_san",
                    f"-Wl,-rpath,{libdir}"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0, (out.returncode, out.stdout, out.stderr)
    assert "c client ok" in out.stdout and "ERROR: AddressSanitizer" not in out.stderr


def test_host_abi_tests_under_asan_ubsan():
    env = dict(os.environ, FLB_LIB=build.LIB_SAN, LD_PRELOAD=build.sanitizer_runtime(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    code = ("import sys, pytest; from paper_1606_07801_amd import flb; "
            "assert flb.LIB_PATH.endswith('libflb_san.so'); "
            "sys.exit(pytest.main(['-q', '-p', 'no:cacheprovider', 'tests/test_abi.py', 'tests/test_layout_host.py']))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600, env=env, cwd=ROOT)
    assert out.returncode == 0, (out.stdout[-3000:], out.stderr[-3000:])
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr
