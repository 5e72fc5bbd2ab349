"""Host-side checks of the C ABI: the library loads, exports what the header declares,
and rejects invalid arguments before touching a device (no GPU needed)."""
import ctypes
import subprocess

import numpy as np
import pytest

import workloads as W
from paper_2305_19768_amd import _abi


@pytest.fixture(scope="module")
def L():
    import __graft_entry__ as g
    g._ensure_built()
    return _abi.lib()


def test_library_exports_every_declared_symbol(L):
    declared = _abi.declared_functions()
    assert {"qmc_plan", "qmc_integrate", "qmc_bind_workspace", "qmc_korobov_search",
            "qmc_lattice_points"} <= set(declared)
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    for f in declared:
        assert hasattr(L, f)
    assert b"gfx950" in L.qmc_version()


def _plan(problem, **kw):
    keep, P = _abi.problem_struct(problem)
    opt = _abi.options_struct(kw.get("m", problem.m), kw.get("precision", 0), 0, kw.get("n_max", 0),
                              kw.get("block", 0), kw.get("shift_tile", 0),
                              kw.get("shifts_per_pass", 0))
    h = ctypes.c_void_p()
    rc = _abi.lib().qmc_plan(ctypes.byref(P), ctypes.byref(opt), ctypes.byref(h))
    return rc, h, keep


def _err():
    return _abi.lib().qmc_last_error().decode()


def test_valid_plan_sizes_workspace_and_frees(L):
    prob = W.two_loop_integral(n_sectors=5, n_scale=0.01)
    rc, h, _ = _plan(prob)
    assert rc == 0, _err()
    nb = L.qmc_workspace_bytes(h)
    assert nb > 0 and nb % 256 == 0
    # integrate before a workspace is bound: state error, nothing launched
    d = ctypes.c_void_p(0x1000)
    assert L.qmc_integrate(h, None, None, None, None, d, d) == -7
    assert "workspace" in _err()
    L.qmc_plan_free(h)
    L.qmc_plan_free(None)


def test_plan_rejects_dimension_beyond_max(L):
    prob = W.two_loop_integral(n_sectors=2, n_scale=0.01)
    keep, P = _abi.problem_struct(prob)
    keep[0][1].d = 9
    opt = _abi.options_struct(prob.m, 0, 0, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    assert L.qmc_plan(ctypes.byref(P), ctypes.byref(opt), ctypes.byref(h)) == -1
    assert "d = 9" in _err()
    keep[0][1].d = 0
    assert L.qmc_plan(ctypes.byref(P), ctypes.byref(opt), ctypes.byref(h)) == -1


@pytest.mark.parametrize("mutate,needle", [
    (lambda s: s.f_exp.__setitem__((1, 0), 4), "degree"),
    (lambda s: s.f_coef.__setitem__(0, np.nan), "non-finite"),
    (lambda s: setattr(s, "transform", "baker") or setattr(s, "f_pow2", 40), "exponent"),
    (lambda s: setattr(s, "integral", 3), "integral"),
])
def test_plan_rejects_invalid_sectors(L, mutate, needle):
    prob = W.two_loop_integral(n_sectors=3, n_scale=0.01)
    mutate(prob.sectors[1])
    rc, h, _ = _plan(prob)
    assert rc == -1 and not h.value
    assert needle in _err()


def test_plan_rejects_invalid_options(L):
    prob = W.one_loop_sector(n=1009)
    assert _plan(prob, m=1)[0] == -1 and "m must be" in _err()
    assert _plan(prob, m=65)[0] == -1
    assert _plan(prob, m=16, shift_tile=17)[0] == -1 and "launch shape" in _err()
    assert _plan(prob, m=16, shift_tile=3)[0] == -1 and "multiple" in _err()
    assert _plan(prob, m=16, shift_tile=16, shifts_per_pass=3)[0] == -1
    assert _plan(prob, m=12, shift_tile=8)[0] == -1 and "multiple" in _err()
    assert _plan(prob, block=96)[0] == -1
    assert _plan(prob, precision=7)[0] == -1
    prob.sectors[0].n = 1
    assert _plan(prob)[0] == -1 and "n_max" in _err()


def test_lattice_points_validates_before_launch(L):
    sh = np.array([0.1, 0.2, 0.3])
    p = sh.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    out = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation
    assert L.qmc_lattice_points(1, 3, 1, p, 0, 1, None, out) == -1
    assert L.qmc_lattice_points(101, 9, 1, p, 0, 1, None, out) == -1
    assert L.qmc_lattice_points(101, 3, 5, p, 100, 2, None, out) == -1 and "outside" in _err()
    assert L.qmc_lattice_points(6, 3, 2, p, 0, 6, None, out) == -1 and "factor" in _err()
    bad = np.array([0.1, 1.0, 0.3])
    assert L.qmc_lattice_points(101, 3, 5, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                0, 5, None, out) == -1
    assert L.qmc_lattice_points(101, 3, 5, p, 0, 0, None, out) == 0   # empty: nothing to do


def test_complex_plan_validation_and_shape(L):
    prob = W.physical_scan(seed=0, n_points=1, n_sectors=2, d_lo=3, d_hi=4, n=1009, m=16)
    rc, h, _ = _plan(prob)
    assert rc == 0, _err()
    assert L.qmc_plan_complex(h) == 1
    # 2 K = 6 columns: the default tile shrinks so that tile * 6 <= 64 (8 of the 16 shifts)
    nb_c = L.qmc_workspace_bytes(h)
    L.qmc_plan_free(h)
    for s in prob.sectors:
        s.deform_lambda = 0.0
    rc, h, _ = _plan(prob)
    assert rc == 0 and L.qmc_plan_complex(h) == 0
    assert L.qmc_workspace_bytes(h) < nb_c
    # real plans refuse deformation calls; no device is touched
    lam = np.array([0.5, 0.5])
    assert L.qmc_set_deformation(h, lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 None) == -7
    assert "real" in _err()
    assert L.qmc_choose_deformation(h, 1009, None, 4, None, None, None) == -7
    assert L.qmc_integrate_deformed(h, None, None, 4, None, None, None, None, None, None) == -7
    assert "real" in _err()
    L.qmc_plan_free(h)
    assert L.qmc_plan_complex(None) == -1
    prob.sectors[1].deform_lambda = -0.5
    assert _plan(prob)[0] == -1 and "deform_lambda" in _err()
    prob.sectors[1].deform_lambda = float("inf")
    assert _plan(prob)[0] == -1
    prob.sectors[1].deform_lambda = 0.5
    assert _plan(prob, shifts_per_pass=2)[0] == -1 and "one shift per pass" in _err()
    assert _plan(prob, shift_tile=16)[0] == -1 and "launch shape" in _err()
    assert _plan(prob, shift_tile=8)[0] == 0


def test_launch_shape_validation(L):
    prob = W.two_loop_integral(n_sectors=2, n_scale=0.01, m=16)
    rc, h, _ = _plan(prob)
    assert rc == 0
    S = _abi.LaunchShape
    assert L.qmc_set_launch_shape(h, ctypes.byref(S(96, 8, 2, 16384, 0))) == -1
    assert L.qmc_set_launch_shape(h, ctypes.byref(S(256, 3, 1, 16384, 0))) == -1
    assert L.qmc_set_launch_shape(h, ctypes.byref(S(256, 8, 3, 16384, 0))) == -1
    assert L.qmc_set_launch_shape(h, ctypes.byref(S(256, 8, 2, 100, 0))) == -1
    assert L.qmc_set_launch_shape(h, ctypes.byref(S(256, 8, 2, 40000, 0))) == -1
    assert L.qmc_set_launch_shape(h, ctypes.byref(S(128, 4, 4, 8192, 0))) == 0
    got = S()
    assert L.qmc_get_launch_shape(h, ctypes.byref(got)) == 0
    assert (got.block, got.shift_tile, got.shifts_per_pass, got.target_blocks) == (128, 4, 4, 8192)
    # timing needs a bound workspace: refused before any device call
    assert L.qmc_autotune(h, None, None, 1, 0, None, None) == -7
    L.qmc_plan_free(h)


def test_flow_shapes_and_sizes(L):
    # parameter counts of (conditional) flows: per layer 64 (d + c) + 64 + 64^2 + 64 + 2d 64 + 2d
    def per(d, c):
        return 4 * (64 * (d + c) + 64 + 64 * 64 + 64 + 2 * d * 64 + 2 * d)
    assert L.qmc_flow_param_count(6, 0) == per(6, 0) == 21552
    assert L.qmc_flow_param_count(6, 2) == per(6, 2)
    assert L.qmc_flow_param_count(8, 4) == per(8, 4)
    for d, c in [(0, 0), (9, 0), (3, 5), (6, -1)]:
        assert L.qmc_flow_param_count(d, c) == -1
        assert L.qmc_flow_bytes(d, c) == 0
    assert L.qmc_flow_bytes(6, 2) > 4 * 4 * per(6, 2)     # params, two moments, gradient, pack
    assert L.qmc_flow_scratch_bytes(6, 2, 0) == 0
