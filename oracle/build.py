"""Compile the plain C oracle into ``oracle/liboracle.so`` (test infrastructure only).

Built with gcc, ``-O2 -ffp-contract=off`` so every fp32 operation of the front
end is one IEEE operation (no fused multiply-add). Every entry point is
single-threaded except ``orc_integrate_omp``, the all-core timing leg
(OpenMP), whose planes equal the single-threaded ones bit for bit.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dbtsdf_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-fopenmp", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
