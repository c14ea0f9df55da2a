"""The C ABI from C: tests/c_client.c is compiled as C99 against
include/flb.h, linked with the built library and run (host-side calls only,
no GPU)."""

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
