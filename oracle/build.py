"""Compile the FP64 oracle (test infrastructure) into oracle/_rara_oracle.so.

Generic x86-64 code, no FMA contraction, so that the oracle's arithmetic is
the plain double-precision sequence written in rara_oracle.c on any host.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rara_oracle.c")
OUT = os.path.join(HERE, "_rara_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-std=c11", "-Wall", "-Wno-unused-variable", SRC, "-o", OUT + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
