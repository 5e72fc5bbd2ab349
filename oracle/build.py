"""Builds the CPU oracle shared object (plain C, FP64, no FMA contraction).

TEST INFRASTRUCTURE ONLY: the oracle checks the HIP library; nothing in the
product path loads it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qmc_oracle.c")
LIB = os.path.join(HERE, "libqmc_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-msse2",
           "-mfpmath=sse", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC,
           "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
