"""Build libaf.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libaf.so")
SOURCES = [os.path.join(CSRC, f) for f in ("af_lib.hip", "af_batch.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("af_device.hpp", "af_kernels.hpp", "af_step.hpp",
                                           "af_host.hpp")] + \
    [os.path.join(ROOT, "include", "af.h")]
ARCH = "gfx950"
# packed FP32 instructions are disabled for all device code
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False, extra=None) -> str:
    cmd = [hipcc()] + FLAGS + list(extra or []) + ["-I", os.path.join(ROOT, "include"),
                                                   "-I", CSRC] + SOURCES + \
        ["-lrocprofiler-sdk-roctx", "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    import sys
    build(verbose=True, extra=sys.argv[1:])
