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


def flags():
    return ["-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-msse2",
            "-mfpmath=sse", "-fPIC", "-shared", "-Wall", "-Wextra"]


def compile_lib(src: str, out: str, verbose: bool = False, extra=None) -> str:
    """Compiles one C source of the oracle to the shared object `out` (atomically)."""
    cmd = ["gcc", *flags(), *(extra or []), "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    return compile_lib(SRC, LIB, verbose)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
