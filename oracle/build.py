"""Compile the CPU oracle (test infrastructure) into ``oracle/liboracle.so``.

Flags: -O2, no FMA contraction and no fast-math, so each operation is rounded
exactly as written; OpenMP only spreads independent grid lines over threads.
``-mfma`` lets the explicit fma() calls of the source run as the processor's
fused multiply-add instruction (the same correctly rounded result as the C
library's software fma, without its cost); contraction stays off, so no
other product and sum is fused.

``build(plain=True)`` compiles the same source with ``-DORC_PLAIN`` into
``liboracle_plain.so``: every explicit product-plus-sum is evaluated with two
roundings.  The tests compare the two builds; nothing else loads it.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wcnst_oracle.c")
LIB_PATH = os.path.join(HERE, "liboracle.so")
PLAIN_LIB_PATH = os.path.join(HERE, "liboracle_plain.so")


def build(plain: bool = False) -> str:
    out = PLAIN_LIB_PATH if plain else LIB_PATH
    tmp = f"{out}.tmp{os.getpid():x}"  # own file: parallel workers may rebuild at once
    cmd = ["gcc", "-O2", "-std=c11", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           *(["-DORC_PLAIN"] if plain else []), "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
    print(build(plain=True))
