"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Flags: -O2 without fast-math and with -ffp-contract=off, so every expression
in pf_oracle.c and pf_oracle_mesh.c rounds exactly as written (round-to-nearest, no FMA fusion,
correctly rounded division and square root).  OpenMP only splits z planes of a
sweep over threads; results do not depend on the thread count.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pf_oracle.c")
SRC_MESH = os.path.join(HERE, "pf_oracle_mesh.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
        "-fno-fast-math", "-fopenmp", "-Wall", "-Wextra", "-o", LIB, SRC, SRC_MESH, "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
        os.path.getmtime(SRC), os.path.getmtime(SRC_MESH),
        os.path.getmtime(os.path.join(HERE, "pf_oracle.h"))
    ):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
