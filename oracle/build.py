"""Build the CPU oracle library (test infrastructure; see bgk_oracle.cpp)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bgk_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build_oracle(force: bool = True, verbose: bool = False) -> str:
    """Compile liboracle.so with g++ (FP64, no fast-math, no FMA contraction)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build_oracle(force=True, verbose=True)
    sys.exit(0)
