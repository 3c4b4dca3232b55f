"""Builds the CPU oracles (test infrastructure): oracle/libensei_oracle.so and
oracle/libensei_bfv_oracle.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ensei_oracle.c")
LIB = os.path.join(HERE, "libensei_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra", SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    # the packed (BFV / RLWE) instantiation's oracle
    from oracle import bfv

    bfv.build(verbose=verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
