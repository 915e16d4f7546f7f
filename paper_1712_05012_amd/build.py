"""Compile libkcm.so (host runtime + gfx950 kernels) in place with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkcm.so")
ARCH = os.environ.get("KCM_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are switched off for all device code.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result"]


def build(verbose: bool = False) -> str:
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["hipcc", *HIP_FLAGS, "-shared", "-o", tmp,
           "-x", "hip", os.path.join(CSRC, "kcm_kernels.hip"),
           "-x", "hip", os.path.join(CSRC, "kcm_host.cpp")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
