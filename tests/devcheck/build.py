"""Builds tests/devcheck/libdevcheck.so (gfx950), the device-arithmetic
check library the GPU tests load."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "wcnst_devcheck.hip")
LIB = os.path.join(HERE, "libdevcheck.so")


def build() -> str:
    csrc = os.path.join(ROOT, "paper_1810_07806_amd", "csrc")
    cmd = [os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "--offload-arch=gfx950", "-O3",
           "-std=c++17", "-fPIC", "-shared", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-ffp-contract=off", "-fno-fast-math", "-I", csrc, "-o", LIB + ".tmp", SRC]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
