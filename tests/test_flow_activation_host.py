"""The flow network's float32 tanh (qmc_flow_kernels.hip, tanh_f), checked on the host:
its coefficients, read from the kernel source, are the ones the committed fit produces,
and the formula evaluated as the kernel evaluates it (float32 fused Horner steps, one
reciprocal) stays within 5e-7 of tanh relative, is odd, and monotone and bounded by 1 up to that error (its rounding wobbles by a few
units of the last place where tanh is close to 1)."""
import importlib.util
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_19768_amd", "csrc")


def _fit_module():
    spec = importlib.util.spec_from_file_location("fit_tanh", os.path.join(CSRC, "fit_tanh.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _kernel_coefficients():
    src = open(os.path.join(CSRC, "qmc_flow_kernels.hip")).read()
    body = src[src.index("float tanh_f(float x)"):]
    body = body[:body.index("\n}\n")]
    lit = r"(0x[0-9a-f.]+p[-+]?\d+|1\.0)f"
    p = [float.fromhex(v) if v.startswith("0x") else 1.0
         for v in re.findall(r"float p = " + lit + r"|fmaf\(p, t, " + lit, body) for v in v if v]
    q = [float.fromhex(v) if v.startswith("0x") else 1.0
         for v in re.findall(r"float q = " + lit + r"|fmaf\(q, t, " + lit, body) for v in v if v]
    clamp = re.search(r"fmed3f\(x, -([0-9.]+)f, ([0-9.]+)f\)", body)
    return p[::-1], q[::-1], float(clamp.group(2))


def test_kernel_coefficients_are_the_fit():
    fit = _fit_module()
    p, q, xmax = _kernel_coefficients()
    assert len(p) == len(q) == fit.DEG + 1 and xmax == fit.XMAX
    pf, qf, err = fit.fit()
    assert err < 3e-8
    assert p == [float(np.float32(v)) for v in pf]
    assert q == [float(np.float32(v)) for v in qf]


def test_float32_evaluation_accuracy_and_shape():
    fit = _fit_module()
    p, q, _ = _kernel_coefficients()
    xs = np.concatenate([np.linspace(-16, 16, 800001), np.geomspace(1e-38, 16, 100001)])
    xs = np.unique(np.concatenate([xs, -xs]).astype(np.float32)).astype(np.float64)
    r = fit.eval_f32(p, q, xs).astype(np.float64)
    ref = np.tanh(xs)
    nz = ref != 0
    assert np.max(np.abs(r[nz] / ref[nz] - 1.0)) < 5e-7
    assert np.all(np.abs(r) <= 1.0 + 5e-7)
    assert np.array_equal(fit.eval_f32(p, q, -xs), -fit.eval_f32(p, q, xs))   # odd
    assert np.all(np.diff(r) >= -1e-6 * np.abs(r[1:]))                          # monotone
    assert fit.eval_f32(p, q, np.array([0.0]))[0] == 0.0
