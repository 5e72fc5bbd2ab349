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


def compile_lib(src: str, out: str, verbose: bool = False, extra=None, cc: str = "gcc") -> str:
    """Compiles one C source of the oracle to the shared object `out` (atomically)."""
    cmd = [cc, *flags(), *(extra or []), "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(verbose: bool = False) -> str:
    return compile_lib(SRC, LIB, verbose)


def build_sanitized(out: str, verbose: bool = False) -> str:
    """The oracle with AddressSanitizer and UndefinedBehaviorSanitizer, compiled by the
    ROCm clang so that it shares one ASan runtime with the sanitized HIP library."""
    cc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")
    return compile_lib(SRC, out, verbose, cc=cc,
                       extra=["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                              "-fno-omit-frame-pointer", "-g"])


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
