"""Compile the CPU oracle (plain C, OpenMP) into oracle/liboracle.so.

Test infrastructure only.  No -ffast-math and no FMA contraction: the oracle's
binary64 arithmetic must be plain IEEE round-to-nearest.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas",
           SRC, "-o", OUT + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
