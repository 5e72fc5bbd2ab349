"""ctypes mirror of include/qmcamp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# QMC_LIBRARY selects another build of the same library (the sanitizer build of the
# host code); the default is the in-tree libqmcamp.so.
LIB_PATH = os.environ.get("QMC_LIBRARY") or os.path.join(HERE, "libqmcamp.so")

QMC_MAX_DIM = 8
QMC_MAX_ORDERS = 4
QMC_MAX_LOG = 4
QMC_PREC_FP64 = 0
QMC_PREC_FP32 = 1
QMC_SPEC_COMPILE_ONLY = 1
QMC_SPEC_OFF = 2
QMC_SPEC_PERSISTENT = 4
TRANSFORMS = {"none": 0, "baker": 1, "korobov1": 2, "korobov2": 3, "korobov3": 4,
              "korobov4": 5, "korobov5": 6, "korobov6": 7}

STATUS_NAMES = {0: "QMC_OK", -1: "QMC_E_INVAL", -2: "QMC_E_NOMEM", -3: "QMC_E_DEVICE",
                -4: "QMC_E_NONFINITE", -5: "QMC_E_TIMEOUT", -6: "QMC_E_SIGNCHECK",
                -7: "QMC_E_STATE"}


class QmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class SectorDesc(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("integral", ctypes.c_int32), ("n_u", ctypes.c_int32),
                ("n_f", ctypes.c_int32), ("u_off", ctypes.c_int64), ("f_off", ctypes.c_int64),
                ("x_pow2", ctypes.c_int32 * QMC_MAX_DIM), ("u_pow", ctypes.c_int32),
                ("f_pow2", ctypes.c_int32), ("transform", ctypes.c_int32),
                ("reserved0", ctypes.c_int32),
                ("logc", (ctypes.c_double * (QMC_MAX_LOG + 1)) * QMC_MAX_ORDERS),
                ("n", ctypes.c_uint64), ("a", ctypes.c_uint64),
                ("deform_lambda", ctypes.c_double)]


class LaunchShape(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("shift_tile", ctypes.c_int32),
                ("shifts_per_pass", ctypes.c_int32), ("target_blocks", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class Problem(ctypes.Structure):
    _fields_ = [("n_sectors", ctypes.c_int32), ("n_orders", ctypes.c_int32),
                ("order_lo", ctypes.c_int32), ("max_log", ctypes.c_int32),
                ("n_integrals", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("sectors", ctypes.POINTER(SectorDesc)),
                ("mono_exp", ctypes.POINTER(ctypes.c_uint8)),
                ("mono_coef", ctypes.POINTER(ctypes.c_double)), ("n_mono_rows", ctypes.c_int64)]


class Options(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("n_max", ctypes.c_uint64), ("block", ctypes.c_int32),
                ("shift_tile", ctypes.c_int32), ("shifts_per_pass", ctypes.c_int32),
                ("reserved0", ctypes.c_int32)]


class Amplitude(ctypes.Structure):
    _fields_ = [("n_sums", ctypes.c_int32), ("n_terms", ctypes.c_int32),
                ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
                ("col", ctypes.POINTER(ctypes.c_int32)),
                ("coef_re", ctypes.POINTER(ctypes.c_double)),
                ("coef_im", ctypes.POINTER(ctypes.c_double)),
                ("coef_order_lo", ctypes.c_int32), ("reserved0", ctypes.c_int32)]


class AmpOptions(ctypes.Structure):
    _fields_ = [("epsrel", ctypes.c_double), ("epsabs", ctypes.c_double),
                ("timeout_s", ctypes.c_double), ("alpha", ctypes.c_double),
                ("n_presample", ctypes.c_uint64), ("max_rounds", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("n_lattice", ctypes.c_int32),
                ("reserved0", ctypes.c_int32),
                ("lattice_n", ctypes.POINTER(ctypes.c_uint64)),
                ("lattice_a", ctypes.POINTER(ctypes.c_uint64)),
                ("tau", ctypes.POINTER(ctypes.c_double)),
                ("tau_used", ctypes.POINTER(ctypes.c_double))]


class AmpStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("timed_out", ctypes.c_int32), ("lattice_limited", ctypes.c_int32),
                ("evaluations", ctypes.c_int64), ("seconds", ctypes.c_double),
                ("max_eps_rel", ctypes.c_double)]


_lib = None


def lib():
    """The loaded libqmcamp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.qmc_plan.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options),
                               ctypes.POINTER(vp)]
        L.qmc_plan.restype = ctypes.c_int
        L.qmc_workspace_bytes.argtypes = [vp]
        L.qmc_workspace_bytes.restype = ctypes.c_size_t
        L.qmc_bind_workspace.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.qmc_bind_workspace.restype = ctypes.c_int
        L.qmc_set_shifts.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp]
        L.qmc_set_shifts.restype = ctypes.c_int
        L.qmc_integrate.argtypes = [vp, u64p, u64p, vp, vp, vp, vp]
        L.qmc_integrate.restype = ctypes.c_int
        L.qmc_query_status.argtypes = [vp, vp, i32p, i32p, i32p]
        L.qmc_query_status.restype = ctypes.c_int
        L.qmc_plan_complex.argtypes = [vp]
        L.qmc_plan_complex.restype = ctypes.c_int32
        L.qmc_sign_violations.argtypes = [vp, vp, u64p]
        L.qmc_sign_violations.restype = ctypes.c_int
        L.qmc_set_deformation.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp]
        L.qmc_set_deformation.restype = ctypes.c_int
        L.qmc_choose_deformation.argtypes = [vp, ctypes.c_uint64, u64p, ctypes.c_int32, vp,
                                             ctypes.POINTER(ctypes.c_double), i32p]
        L.qmc_choose_deformation.restype = ctypes.c_int
        L.qmc_integrate_deformed.argtypes = [vp, u64p, u64p, ctypes.c_int32, vp, vp, vp, vp,
                                             ctypes.POINTER(ctypes.c_double), i32p]
        L.qmc_integrate_deformed.restype = ctypes.c_int
        L.qmc_integrate_static.argtypes = [vp, u64p, u64p, vp, vp, vp, vp]
        L.qmc_integrate_static.restype = ctypes.c_int
        L.qmc_integrate_vec.argtypes = [vp, u64p, u64p, vp, vp, vp, vp]
        L.qmc_integrate_vec.restype = ctypes.c_int
        L.qmc_median_workspace_bytes.argtypes = [vp, ctypes.c_int32]
        L.qmc_median_workspace_bytes.restype = ctypes.c_size_t
        L.qmc_median_lattice.argtypes = [vp, u64p, ctypes.c_int32, u64p, ctypes.c_int32, vp,
                                         ctypes.c_size_t, vp, u64p, ctypes.POINTER(ctypes.c_double)]
        L.qmc_median_lattice.restype = ctypes.c_int
        L.qmc_set_launch_shape.argtypes = [vp, ctypes.POINTER(LaunchShape)]
        L.qmc_set_launch_shape.restype = ctypes.c_int
        L.qmc_get_launch_shape.argtypes = [vp, ctypes.POINTER(LaunchShape)]
        L.qmc_get_launch_shape.restype = ctypes.c_int
        L.qmc_autotune.argtypes = [vp, u64p, u64p, ctypes.c_int32, ctypes.c_int32, vp,
                                   ctypes.POINTER(LaunchShape)]
        L.qmc_autotune.restype = ctypes.c_int
        L.qmc_specialize.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        L.qmc_specialize.restype = ctypes.c_int
        L.qmc_gen_source.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p,
                                     ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        L.qmc_gen_source.restype = ctypes.c_int
        from . import flow as _flow
        _flow.bind(L)
        L.qmc_korobov_p2.argtypes = [vp, ctypes.c_uint64, ctypes.c_int32, u64p, ctypes.c_int32,
                                     vp, vp]
        L.qmc_korobov_p2.restype = ctypes.c_int
        L.qmc_korobov_search.argtypes = [vp, ctypes.c_uint64, ctypes.c_int32, u64p,
                                         ctypes.c_int32, vp, u64p,
                                         ctypes.POINTER(ctypes.c_double)]
        L.qmc_korobov_search.restype = ctypes.c_int
        L.qmc_lattice_points.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint64,
                                         ctypes.POINTER(ctypes.c_double), ctypes.c_uint64,
                                         ctypes.c_uint64, vp, vp]
        L.qmc_lattice_points.restype = ctypes.c_int
        L.amp_evaluate.argtypes = [vp, ctypes.POINTER(Amplitude), ctypes.POINTER(AmpOptions), vp,
                                   ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), u64p,
                                   ctypes.POINTER(AmpStats)]
        L.amp_evaluate.restype = ctypes.c_int
        L.qmc_enable_timing.argtypes = [vp, ctypes.c_int32]
        L.qmc_enable_timing.restype = ctypes.c_int
        L.qmc_read_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32p]
        L.qmc_read_timing.restype = ctypes.c_int
        L.qmc_plan_free.argtypes = [vp]
        L.qmc_plan_free.restype = None
        L.qmc_last_error.argtypes = []
        L.qmc_last_error.restype = ctypes.c_char_p
        L.qmc_version.argtypes = []
        L.qmc_version.restype = ctypes.c_char_p
        cpp = ctypes.POINTER(ctypes.c_char_p)
        L.qmc_coef_series.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int32, cpp, cpp,
                                      ctypes.c_int32, ctypes.c_int32, i32p,
                                      ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
        L.qmc_coef_series.restype = ctypes.c_int
        _lib = L
    return _lib


def problem_struct(problem):
    """Packs a workloads.Problem into the C structs; returns (keepalive, Problem)."""
    secs = problem.sectors
    S = len(secs)
    K = problem.K
    M = problem.M
    rows_e, rows_c = [], []
    rows = 0   # monomial rows packed so far
    desc = (SectorDesc * S)()
    for s, sec in enumerate(secs):
        d = int(sec.d)
        D = desc[s]
        D.d = d
        D.integral = int(sec.integral)
        D.n_u = len(sec.u_coef)
        D.n_f = len(sec.f_coef)
        D.u_off = rows
        ue = np.zeros((len(sec.u_coef), QMC_MAX_DIM), dtype=np.uint8)
        ue[:, :d] = np.asarray(sec.u_exp, dtype=np.uint8).reshape(-1, d)
        rows_e.append(ue)
        rows_c.append(np.asarray(sec.u_coef, dtype=np.float64))
        rows += len(rows_c[-1])
        D.f_off = rows
        fe = np.zeros((len(sec.f_coef), QMC_MAX_DIM), dtype=np.uint8)
        fe[:, :d] = np.asarray(sec.f_exp, dtype=np.uint8).reshape(-1, d)
        rows_e.append(fe)
        rows_c.append(np.asarray(sec.f_coef, dtype=np.float64))
        rows += len(rows_c[-1])
        xp = np.zeros(QMC_MAX_DIM, dtype=np.int32)
        xp[:d] = np.asarray(sec.x_pow2, dtype=np.int32)
        for j in range(QMC_MAX_DIM):
            D.x_pow2[j] = int(xp[j])
        D.u_pow = int(sec.u_pow)
        D.f_pow2 = int(sec.f_pow2)
        D.transform = TRANSFORMS[sec.transform]
        lc = np.asarray(sec.logc, dtype=np.float64)
        for k in range(lc.shape[0]):
            for m in range(lc.shape[1]):
                D.logc[k][m] = float(lc[k, m])
        D.n = int(sec.n)
        D.a = int(sec.a)
        D.deform_lambda = float(getattr(sec, "deform_lambda", 0.0))
    exps = np.ascontiguousarray(np.concatenate(rows_e, axis=0) if rows_e else
                                np.zeros((0, QMC_MAX_DIM), np.uint8))
    coef = np.ascontiguousarray(np.concatenate(rows_c) if rows_c else np.zeros(0))
    P = Problem()
    P.n_sectors = S
    P.n_orders = K
    P.order_lo = int(problem.order_lo)
    P.max_log = M
    P.n_integrals = int(getattr(problem, "n_integrals", 1))
    P.sectors = ctypes.cast(desc, ctypes.POINTER(SectorDesc))
    P.mono_exp = exps.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    P.mono_coef = coef.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    P.n_mono_rows = len(coef)
    return (desc, exps, coef), P


def options_struct(m, precision, seed, n_max, block, shift_tile, shifts_per_pass):
    o = Options()
    o.m = int(m)
    o.precision = int(precision)
    o.seed = int(seed) & (2 ** 64 - 1)
    o.n_max = int(n_max)
    o.block = int(block)
    o.shift_tile = int(shift_tile)
    o.shifts_per_pass = int(shifts_per_pass)
    return o


def declared_functions(header=None):
    """Names of the functions include/qmcamp.h declares."""
    import re
    header = header or os.path.join(HERE, "..", "include", "qmcamp.h")
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(qmc_[a-z_0-9]+|amp_[a-z_0-9]+)\s*\(",
                                 text, flags=re.M)))
