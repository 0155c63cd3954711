"""Compile the C brute-force oracle into oracle/liboracle.so (gcc, OpenMP).

Test infrastructure only. Flags: -ffp-contract=off and no -march option, so
the compiler never fuses a multiply and an add; -O2 keeps IEEE semantics
(no -ffast-math).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sj_oracle.c")
GRID_SRC = os.path.join(HERE, "cpu_grid_join.c")  # host-core grid-join baseline
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", SRC, GRID_SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
