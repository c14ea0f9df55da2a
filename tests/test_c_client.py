"""The C ABI from C: tests/c_client.c is compiled as C99 against
include/flb.h, linked with the built library and run: host-side calls
without a GPU, and (GPU test) a lattice created, stepped and read from C."""

import os
import shutil
import subprocess

import pytest

from paper_1606_07801_amd import flb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_c_client(tmp_path):
    libdir = os.path.dirname(flb.LIB_PATH)
    assert os.path.exists(flb.LIB_PATH), "build the library first"
    exe = str(tmp_path / "c_client")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_client.c"), "-o", exe, "-L", libdir, "-lflb",
                    f"-Wl,-rpath,{libdir}"], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, (out.returncode, out.stdout, out.stderr)
    assert "c client ok" in out.stdout


@pytest.mark.gpu
@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_c_client_drives_the_gpu(tmp_path):
    libdir = os.path.dirname(flb.LIB_PATH)
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    exe = str(tmp_path / "c_client_gpu")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-DFLB_CLIENT_GPU", "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(rocm, "include"),
                    os.path.join(ROOT, "tests", "c_client.c"), "-o", exe, "-L", libdir, "-lflb",
                    "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm",
                    f"-Wl,-rpath,{libdir}", f"-Wl,-rpath,{os.path.join(rocm, 'lib')}"], check=True)
    out = subprocess.run([exe, "gpu"], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, (out.returncode, out.stdout, out.stderr)
    assert "c client gpu ok" in out.stdout
