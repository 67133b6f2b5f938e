"""Compile the CPU oracle (test infrastructure) into ``oracle/liboracle.so``.

Flags: -O2, no FMA contraction and no fast-math, so each operation is rounded
exactly as written; OpenMP only spreads independent grid lines over threads.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wcnst_oracle.c")
LIB_PATH = os.path.join(HERE, "liboracle.so")


def build() -> str:
    tmp = f"{LIB_PATH}.tmp{os.getpid():x}"  # own file: parallel workers may rebuild at once
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build())
