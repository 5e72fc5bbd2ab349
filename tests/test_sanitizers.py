"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds a copy of the library whose host sources (planner and table packing, adaptive
loop, flow driver, coefficient-expression parser, code generator) are instrumented,
and the oracle likewise, then runs the host-side test files in a child Python that
preloads the ROCm clang's ASan runtime and loads those copies.  Any sanitizer report
aborts the child (halt_on_error), so the test passes only on a clean run.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# host-side suites: every C-ABI entry that runs without a device, the generated-source
# interpreter, the exact coefficient series (random and malformed strings), the oracle
HOST_SUITES = ["tests/test_abi_host.py", "tests/test_gen_host.py", "tests/test_oracle_coef.py",
               "tests/test_oracle_pins.py", "tests/test_oracle_adaptive.py"]


@pytest.mark.slow
def test_host_code_clean_under_asan_and_ubsan(tmp_path):
    from paper_2305_19768_amd import build as hb
    from oracle import build as ob
    lib = hb.build_sanitized(str(tmp_path / "libqmcamp_asan.so"))
    olib = ob.build_sanitized(str(tmp_path / "libqmc_oracle_asan.so"))
    env = dict(os.environ)
    env.update({
        "QMC_LIBRARY": lib, "QMC_ORACLE_LIBRARY": olib,
        "LD_PRELOAD": hb.asan_runtime(),
        "ASAN_OPTIONS": f"detect_leaks=0:halt_on_error=1:log_path={tmp_path}/asan",
        "UBSAN_OPTIONS": f"halt_on_error=1:print_stacktrace=1:log_path={tmp_path}/ubsan",
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *HOST_SUITES], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=1200)
    reports = sorted(p for p in os.listdir(tmp_path) if p.startswith(("asan", "ubsan")))
    text = "".join(open(tmp_path / p).read()[:4000] for p in reports)
    assert r.returncode == 0 and not reports, (r.stdout[-3000:] + r.stderr[-2000:] + text)
