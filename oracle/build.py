"""Compile the C oracle (oracle/core.c) into oracle/_orc_core.so with gcc.

TEST INFRASTRUCTURE ONLY.  Plain gcc, OpenMP over independent rows, no fast
math and no floating-point contraction (the double-double reference relies on
exactly rounded additions).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "core.c")
LIB = os.path.join(HERE, "_orc_core.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
           SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
