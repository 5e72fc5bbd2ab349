"""Builds libqmcamp.so (HIP kernels for gfx950 + host planner / C ABI) in-tree with hipcc."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqmcamp.so")
SOURCES = ["qmc_kernels.hip", "qmc_amp_kernels.hip", "qmc_deform_kernels.hip",
           "qmc_flow_kernels.hip", "qmc_api.cpp", "qmc_amp.cpp", "qmc_flow.cpp",
           "qmc_coef.cpp"]
ARCH = os.environ.get("QMC_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"),
              shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-result",
            # no packed FP32 math: write only scalar FP32/FP64 arithmetic
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(HERE, "..", "include")]


def build(verbose: bool = False, extra=None) -> str:
    """Compiles every source to an object (in parallel), then links the shared library."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        jobs.append(([hipcc(), *flags(), *(extra or []), "-c", "-o", obj,
                      os.path.join(CSRC, src)], obj))
    if verbose:
        for cmd, _ in jobs:
            print(" ".join(cmd), flush=True)
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        for r in ex.map(lambda j: subprocess.run(j[0], capture_output=True, text=True), jobs):
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise subprocess.CalledProcessError(r.returncode, r.args)
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-o", LIB + ".tmp",
            *[o for _, o in jobs]]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def asm(out_dir: str) -> None:
    """Writes the gfx950 assembly of the kernels (for register and instruction counts)."""
    os.makedirs(out_dir, exist_ok=True)
    cmd = [hipcc(), *flags(), "--cuda-device-only", "-S", "-o",
           os.path.join(out_dir, "qmc_kernels.s"), os.path.join(CSRC, "qmc_kernels.hip")]
    subprocess.run(cmd, check=True)


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "--asm":
        asm(sys.argv[2])
    else:
        build(verbose=True)
