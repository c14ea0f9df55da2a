"""Build the HIP library libflb.so for gfx950 in-tree.

    python -m paper_1606_07801_amd.build [--sanitize]

compiles every .hip source under csrc/ with hipcc into lib/libflb.so.
--sanitize builds lib/libflb_san.so instead, whose host code carries
AddressSanitizer and UndefinedBehaviorSanitizer (the device code is built
as usual); a process using it needs the clang ASan runtime preloaded
(sanitizer_runtime() names it), for the host-side checks on the CPU.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libflb.so")
LIB_SAN = os.path.join(LIBDIR, "libflb_san.so")
# sanitizers on the host side only (GPU code is never built with them)
SAN_FLAGS = ["-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
             "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined"]
ARCH = os.environ.get("FLB_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    # roctx ranges around the API calls (rocprofv3 --marker-trace)
    "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def sanitizer_runtime():
    """The clang ASan runtime of the ROCm toolchain (to LD_PRELOAD)."""
    import glob
    found = sorted(glob.glob(os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "lib", "clang", "*",
                                          "lib", "linux", "libclang_rt.asan-x86_64.so")))
    return found[-1] if found else None


def build(verbose=True, sanitize=False):
    os.makedirs(LIBDIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = LIB_SAN if sanitize else LIB
    tmp = out + ".tmp"
    cmd = [hipcc, *FLAGS, *(SAN_FLAGS if sanitize else []), "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libflb.so")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(sanitize="--sanitize" in sys.argv[1:])
