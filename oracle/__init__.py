"""CPU oracle for randomized rank-1 lattice QMC of sector integrands and amplitudes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_2305_19768_amd``); both consume the seeded arrays of
``workloads`` and nothing else.

Heavy loops live in ``qmc_oracle.c`` (plain scalar C, FP64, Neumaier sums, no FMA
contraction).  The statistics and the lattice-size allocation are written out here
in numpy, each following the passage of arXiv:2305.19768 named in its docstring.

Parity status of each function (what pins it, in ``tests/test_oracle_pins.py``):
  points            lattice identities (permutation columns, z_1 = 1) and exactness on
                    trigonometric polynomials (character-sum identity)
  transform         closed-form properties (phi(0), phi(1), symmetry, phi' = w, int w = 1)
  integrand/sums    closed-form integrals (1-loop massless bubble log^m F moments, separable
                    and mixed-monomial integrals with known values), Gauss-Legendre in 1-3 D,
                    convergence order
  neumaier          exact results of ill-conditioned sums
  p2                truncated dual-lattice sum on small n, Korobov-space identities
  estimate/amplitude/eps_rel  textbook mean/variance, propagation of independent variances
  allocate          constraint + stationarity residuals, brute-force constrained minimum
  amplitude_series  Cauchy product of Laurent series (numpy convolution), Monte-Carlo
                    variance of independent orders, reduction to constant coefficients
  median_rule       brute force over the candidates (test_oracle_pins.py)
  deformed contour  (sector_sums_deformed, integrand_deformed, choose_lambda) closed-form
                    timelike bubble, Cauchy invariance at Euclidean points, lambda = 0
                    branch (test_oracle_deform.py)
  coef.py           exact rational functions, closed-form series, float(Fraction)
                    rounding (test_oracle_coef.py)
  flow.py           identity, invertibility, finite differences, Gauss-Legendre
                    unbiasedness, conditional reduction (test_oracle_flow.py)
"""

from __future__ import annotations

import ctypes
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# QMC_ORACLE_LIBRARY selects another build of the oracle (the sanitizer build)
_LIB_PATH = os.environ.get("QMC_ORACLE_LIBRARY") or os.path.join(_HERE, "libqmc_oracle.so")
_lib = None

TRANSFORM_CODES = {"none": 0, "baker": 1, "korobov1": 2, "korobov2": 3, "korobov3": 4,
                   "korobov4": 5, "korobov5": 6, "korobov6": 7}

_dp = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_points.argtypes = [ctypes.c_uint64, ctypes.c_int, _u64p, _dp, ctypes.c_uint64,
                                ctypes.c_uint64, _dp]
        L.or_points.restype = None
        L.or_transform.argtypes = [ctypes.c_int, ctypes.c_uint64, _dp, _dp, _dp]
        L.or_transform.restype = None
        L.or_integrand.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp, ctypes.c_int, _u8p,
                                   _dp, _i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, _dp, ctypes.c_uint64, _dp, _dp]
        L.or_integrand.restype = ctypes.c_int
        L.or_sums.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp, ctypes.c_int, _u8p, _dp,
                              _i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              _dp, ctypes.c_int, ctypes.c_uint64, _u64p, _dp, ctypes.c_int,
                              ctypes.c_int, _dp, _dp, _i64p]
        L.or_sums.restype = ctypes.c_int
        L.or_neumaier.argtypes = [_dp, ctypes.c_uint64]
        L.or_neumaier.restype = ctypes.c_double
        L.or_p2.argtypes = [ctypes.c_uint64, ctypes.c_int, _u64p]
        L.or_p2.restype = ctypes.c_double
        L.or_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.or_splitmix64.restype = ctypes.c_uint64
        L.or_deform_point.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp, ctypes.c_double,
                                      _dp, _dp, _dp, _dp]
        L.or_deform_point.restype = None
        L.or_sums_deformed.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp, ctypes.c_int,
                                       _u8p, _dp, _i32p, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_uint64, _u64p, _dp, ctypes.c_int,
                                       ctypes.c_int, _dp, _dp, _i64p, _i64p]
        L.or_sums_deformed.restype = ctypes.c_int
        L.or_integrand_deformed.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp, ctypes.c_int,
                                            _u8p, _dp, _i32p, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double,
                                            ctypes.c_uint64, _dp, _dp, _i32p]
        L.or_integrand_deformed.restype = ctypes.c_int
        L.or_sign_violations.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _dp, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_uint64, _u64p, _dp, ctypes.c_int,
                                         ctypes.c_int]
        L.or_sign_violations.restype = ctypes.c_int64
        _lib = L
    return _lib


def _p(a, typ):
    return a.ctypes.data_as(typ)


# ------------------------------------------------------------------ lattice

def korobov_vector(n: int, a: int, d: int) -> np.ndarray:
    """Korobov generating vector z = (1, a, a^2, ..., a^(d-1)) mod n."""
    return np.array([pow(int(a), j, int(n)) for j in range(d)], dtype=np.uint64)


def points(n: int, z: Sequence[int], delta: Sequence[float], i0: int = 0,
           count: Optional[int] = None) -> np.ndarray:
    """Shifted lattice points y_i = frac(i z / n + Delta), i = i0 .. i0+count-1.

    Rank-1 lattice rule of the paper's Sec. 2.2 (definition of Q_{n,z}); k_j = i z_j mod n
    is exact, q_j = k_j / n is the IEEE quotient, the shift wraps by one exact subtraction.
    """
    z = np.ascontiguousarray(z, dtype=np.uint64)
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    d = len(z)
    count = n - i0 if count is None else count
    out = np.empty((count, d), dtype=np.float64)
    lib().or_points(n, d, _p(z, _u64p), _p(delta, _dp), i0, count, _p(out, _dp))
    return out


def transform(kind: str, y) -> tuple:
    """Periodizing transform x = phi(y) and its derivative w = phi'(y), per coordinate."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    x = np.empty_like(y)
    w = np.empty_like(y)
    lib().or_transform(TRANSFORM_CODES[kind], y.size, _p(y, _dp), _p(x, _dp), _p(w, _dp))
    return x, w


class _SectorArrays:
    """Contiguous copies of a sector's tables, kept alive across C calls."""

    def __init__(self, sec):
        self.d = int(sec.d)
        self.u_exp = np.ascontiguousarray(sec.u_exp, dtype=np.uint8).reshape(-1)
        self.u_coef = np.ascontiguousarray(sec.u_coef, dtype=np.float64)
        self.f_exp = np.ascontiguousarray(sec.f_exp, dtype=np.uint8).reshape(-1)
        self.f_coef = np.ascontiguousarray(sec.f_coef, dtype=np.float64)
        self.x_pow2 = np.ascontiguousarray(sec.x_pow2, dtype=np.int32)
        self.logc = np.ascontiguousarray(sec.logc, dtype=np.float64)
        self.K, self.M = self.logc.shape[0], self.logc.shape[1] - 1
        self.n_u, self.n_f = len(self.u_coef), len(self.f_coef)
        self.u_pow, self.f_pow2 = int(sec.u_pow), int(sec.f_pow2)
        self.transform = TRANSFORM_CODES[sec.transform]

    def head(self):
        return (self.d, self.n_u, _p(self.u_exp, _u8p), _p(self.u_coef, _dp), self.n_f,
                _p(self.f_exp, _u8p), _p(self.f_coef, _dp), _p(self.x_pow2, _i32p),
                self.u_pow, self.f_pow2, self.K, self.M, _p(self.logc, _dp))


def integrand(sec, x) -> np.ndarray:
    """f_k(x) = x^p U^a F^b sum_m c_{k,m} (log F)^m for each order k, at points x [count, d]."""
    A = _SectorArrays(sec)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, A.d)
    out = np.empty((x.shape[0], A.K), dtype=np.float64)
    lib().or_integrand(*A.head(), x.shape[0], _p(x, _dp), _p(out, _dp))
    return out


class OracleNonFinite(RuntimeError):
    pass


class OracleSignCheck(RuntimeError):
    pass


def sector_sums(sec, shifts, n: Optional[int] = None, a: Optional[int] = None,
                z: Optional[Sequence[int]] = None, shift_range=None, threads: int = 1):
    """Per-shift lattice estimates of one sector.

    Returns (Q, S) with Q[l, k] = (1/n) sum_i W f_k and S[l, k] = (1/n) sum_i |W f_k|,
    summed with Neumaier compensation (the per-shift sums of Sec. 2.1).  A sector with
    deform_lambda > 0 is integrated on the deformed contour: Q is complex and a failed
    sign check raises OracleSignCheck (use sector_sums_deformed for the counts).
    """
    if getattr(sec, "deform_lambda", 0.0) > 0.0:
        Q, S, viol, first = sector_sums_deformed(sec, shifts, n=n, a=a, z=z,
                                                 shift_range=shift_range, threads=threads)
        if viol:
            raise OracleSignCheck(f"Im F(z) > 0 at {viol} samples, first (shift, index) {first}")
        return Q, S
    A = _SectorArrays(sec)
    n = int(sec.n if n is None else n)
    if z is None:
        z = korobov_vector(n, sec.a if a is None else a, A.d)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    shifts = np.ascontiguousarray(shifts, dtype=np.float64)
    m = shifts.shape[0]
    l0, l1 = (0, m) if shift_range is None else shift_range
    Q = np.empty((l1 - l0, A.K))
    S = np.empty((l1 - l0, A.K))
    L = lib()

    def run(lo, hi):
        bad = np.zeros(2, dtype=np.int64)
        q = np.empty((hi - lo, A.K))
        s = np.empty((hi - lo, A.K))
        rc = L.or_sums(*A.head(), A.transform, n, _p(z, _u64p), _p(shifts, _dp), lo, hi,
                       _p(q, _dp), _p(s, _dp), _p(bad, _i64p))
        if rc == 1:
            raise OracleNonFinite(f"non-finite sample at shift {bad[0]}, index {bad[1]}")
        if rc != 0:
            raise ValueError("invalid sector")
        Q[lo - l0:hi - l0] = q
        S[lo - l0:hi - l0] = s

    if threads <= 1 or l1 - l0 == 1:
        run(l0, l1)
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(lambda l: run(l, l + 1), range(l0, l1)))
    return Q, S


def deform_point(sec, x, lam: Optional[float] = None):
    """z(x), J(x) = det dz/dx and F(z) of the deformed contour at real points x [count, d]
    (z_j = x_j - i lambda x_j (1 - x_j) dF/dx_j)."""
    A = _SectorArrays(sec)
    lam = float(sec.deform_lambda if lam is None else lam)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, A.d)
    z = np.empty((x.shape[0], A.d, 2))
    J = np.empty((x.shape[0], 2))
    F = np.empty((x.shape[0], 2))
    for t in range(x.shape[0]):
        xt = np.ascontiguousarray(x[t])
        zt, Jt, Ft = np.empty((A.d, 2)), np.empty(2), np.empty(2)
        lib().or_deform_point(A.d, A.n_f, _p(A.f_exp, _u8p), _p(A.f_coef, _dp), lam,
                              _p(xt, _dp), _p(zt, _dp), _p(Jt, _dp), _p(Ft, _dp))
        z[t], J[t], F[t] = zt, Jt, Ft
    return (z[..., 0] + 1j * z[..., 1], J[:, 0] + 1j * J[:, 1], F[:, 0] + 1j * F[:, 1])


def integrand_deformed(sec, x, lam: Optional[float] = None):
    """J(x) f_k(z(x)) on the deformed contour at real points x [count, d] (complex
    [count, K]) and whether each sample violates the sign check (bool [count])."""
    A = _SectorArrays(sec)
    lam = float(sec.deform_lambda if lam is None else lam)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, A.d)
    out = np.empty((x.shape[0], A.K, 2))
    viol = np.empty(x.shape[0], dtype=np.int32)
    rc = lib().or_integrand_deformed(*A.head(), lam, x.shape[0], _p(x, _dp), _p(out, _dp),
                                     _p(viol, _i32p))
    if rc != 0:
        raise ValueError("invalid sector")
    return out[..., 0] + 1j * out[..., 1], viol.astype(bool)


def sector_sums_deformed(sec, shifts, n: Optional[int] = None, a: Optional[int] = None,
                         z: Optional[Sequence[int]] = None, shift_range=None, threads: int = 1,
                         lam: Optional[float] = None):
    """Per-shift estimates of one sector on the deformed contour.

    Returns (Q complex [l, k], S [l, k] = (1/n) sum |W J f_k|, number of samples with
    Im F(z) > 0, (shift, index) of the first such sample or None)."""
    A = _SectorArrays(sec)
    lam = float(sec.deform_lambda if lam is None else lam)
    n = int(sec.n if n is None else n)
    if z is None:
        z = korobov_vector(n, sec.a if a is None else a, A.d)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    shifts = np.ascontiguousarray(shifts, dtype=np.float64)
    m = shifts.shape[0]
    l0, l1 = (0, m) if shift_range is None else shift_range
    Q = np.empty((l1 - l0, A.K), dtype=np.complex128)
    S = np.empty((l1 - l0, A.K))
    sign = np.zeros((l1 - l0, 3), dtype=np.int64)
    L = lib()

    def run(l):
        bad = np.zeros(2, dtype=np.int64)
        sg = np.zeros(3, dtype=np.int64)
        q = np.empty((1, A.K, 2))
        s = np.empty((1, A.K))
        rc = L.or_sums_deformed(*A.head(), lam, A.transform, n, _p(z, _u64p), _p(shifts, _dp),
                                l, l + 1, _p(q, _dp), _p(s, _dp), _p(bad, _i64p),
                                _p(sg, _i64p))
        if rc == 1:
            raise OracleNonFinite(f"non-finite sample at shift {bad[0]}, index {bad[1]}")
        if rc != 0:
            raise ValueError("invalid sector")
        Q[l - l0] = q[0, :, 0] + 1j * q[0, :, 1]
        S[l - l0] = s[0]
        sign[l - l0] = sg

    if threads <= 1 or l1 - l0 == 1:
        for l in range(l0, l1):
            run(l)
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(run, range(l0, l1)))
    viol = int(sign[:, 0].sum())
    first = None
    for row in sign:
        if row[0] > 0:
            first = (int(row[1]), int(row[2]))
            break
    return Q, S, viol, first


def sign_violations(sec, shifts, lam: float, n: int, a: int) -> int:
    """Samples of the lattice (n, Korobov a) and the given shifts with Im F(z) > 0."""
    A = _SectorArrays(sec)
    z = korobov_vector(n, a, A.d)
    shifts = np.ascontiguousarray(shifts, dtype=np.float64)
    return int(lib().or_sign_violations(A.d, A.n_f, _p(A.f_exp, _u8p), _p(A.f_coef, _dp),
                                        float(lam), A.transform, int(n), _p(z, _u64p),
                                        _p(shifts, _dp), 0, shifts.shape[0]))


def choose_lambda(sec, shifts, lam0: float, n: int, a: int, max_halvings: int = 16):
    """Deformation parameter from presamples (the library-call parameter
    number_of_presamples of Sec. 3.1.3): start at lam0 and halve until no presample
    point has Im F(z) > 0.  Returns (lambda, halvings) or raises OracleSignCheck."""
    lam = float(lam0)
    for h in range(max_halvings + 1):
        if sign_violations(sec, shifts, lam, n, a) == 0:
            return lam, h
        lam *= 0.5
    raise OracleSignCheck(f"no valid deformation parameter down to {lam * 2:g}")


def median_rule(sec, n: int, candidates, order: int = -1):
    """Median QMC rule (Sec. 2.2, Eq. median): the unshifted rank-1 lattice estimates
    Q_{n,z_c} of candidates z_c [r, d] (components in U_n), and the candidate whose
    estimate of epsilon order `order` is the median (r odd: the middle one; r even: the
    lower middle; equal estimates ordered by candidate index).
    Returns (chosen index, Q [r, K])."""
    cands = np.ascontiguousarray(candidates, dtype=np.uint64).reshape(-1, sec.d)
    zero = np.zeros((1, sec.d))
    Q = np.empty((cands.shape[0], sec.K))
    for c, z in enumerate(cands):
        Q[c] = sector_sums(sec, zero, n=n, z=z)[0][0]
    key = Q[:, order]
    idx = sorted(range(len(key)), key=lambda c: (key[c], c))
    return idx[(len(idx) - 1) // 2], Q


def problem_sums(problem, threads: int = 1, sectors=None):
    """Q[s] (m x K) and S[s] for every sector of a workloads.Problem."""
    idx = range(len(problem.sectors)) if sectors is None else sectors
    out_q, out_s = [], []
    for s in idx:
        sec = problem.sectors[s]
        q, a = sector_sums(sec, problem.shifts[s], threads=threads)
        out_q.append(q)
        out_s.append(a)
    return out_q, out_s


def neumaier(v) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().or_neumaier(_p(v, _dp), v.size)


def splitmix64(seed: int, counter: int) -> int:
    return int(lib().or_splitmix64(seed & (2**64 - 1), counter & (2**64 - 1)))


def seeded_shifts(seed: int, sector: int, m: int, d: int) -> np.ndarray:
    """Shift Delta_{s,l,j} = (splitmix64(seed, (s << 32) | (l << 8) | j) >> 11) * 2^-53."""
    out = np.empty((m, d))
    for l in range(m):
        for j in range(d):
            c = (sector << 32) | (l << 8) | j
            out[l, j] = (splitmix64(seed, c) >> 11) * 2.0 ** -53
    return out


# ---------------------------------------------------------------- P_2 search

def p2(n: int, z: Sequence[int]) -> float:
    """P_2 figure of merit (Korobov space, alpha = 2, unit product weights; Sec. 2.2)."""
    z = np.ascontiguousarray(z, dtype=np.uint64)
    return float(lib().or_p2(n, len(z), _p(z, _u64p)))


def korobov_search(n: int, d: int, candidates: Sequence[int], rel_tie: float = 1e-12,
                   threads: int = 1):
    """Korobov parameter a minimising P_2 over the candidates.

    Candidates within a relative rel_tie of the minimum count as tied and the smallest
    a wins (P_2(a) = P_2(n - a) and P_2 is invariant under coordinate reversal, so exact
    ties are common).  Returns (a, p2 values).
    """
    cands = [int(c) for c in candidates]

    def f(a):
        return p2(n, korobov_vector(n, a, d))

    if threads > 1:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            vals = list(ex.map(f, cands))
    else:
        vals = [f(a) for a in cands]
    vmin = min(vals)
    tied = [a for a, v in zip(cands, vals) if v <= vmin * (1.0 + rel_tie)]
    return min(tied), np.array(vals)


# --------------------------------------------------------------- statistics

def estimate(Q):
    """Mean over the m shift estimates and its standard error sqrt(var/m), var unbiased.

    Error from the shifts as in the caption of the precision-by-lattice figure (Sec. 2.1.3).
    Q has shape [m, ...]; returns (mean, err) of shape [...].
    """
    Q = np.asarray(Q, dtype=np.float64)
    m = Q.shape[0]
    mean = Q.sum(axis=0) / m
    var = ((Q - mean) ** 2).sum(axis=0) / (m - 1)
    return mean, np.sqrt(var / m)


def integral_values(problem, means: List[np.ndarray], errs: List[np.ndarray]):
    """Integral I_c = sum of its sectors; variances of independent sectors add."""
    K = problem.K
    val = np.zeros((problem.n_integrals, K))
    var = np.zeros((problem.n_integrals, K))
    for s, sec in enumerate(problem.sectors):
        val[sec.integral] += means[s]
        var[sec.integral] += errs[s] ** 2
    return val, np.sqrt(var)


def amplitude(coef, ival, ierr, ival_im=None, ierr_im=None):
    """A_k = sum_i C_i I_{i,k} with var(A_k) = sum_i |C_i|^2 var(I_{i,k}) (Sec. 2.1.3, Eq. 4).

    For complex C and I, Re and Im of each integral are independent, so
    var(Re A) = sum (Re C)^2 var(Re I) + (Im C)^2 var(Im I) and likewise for Im A.
    Returns (re, im, err_re, err_im), each of shape [K].
    """
    C = np.asarray(coef, dtype=np.complex128)
    ir = np.asarray(ival, dtype=np.float64)
    ii = np.zeros_like(ir) if ival_im is None else np.asarray(ival_im, dtype=np.float64)
    er = np.asarray(ierr, dtype=np.float64)
    ei = np.zeros_like(er) if ierr_im is None else np.asarray(ierr_im, dtype=np.float64)
    cr, ci = C.real[:, None], C.imag[:, None]
    re = (cr * ir - ci * ii).sum(axis=0)
    im = (cr * ii + ci * ir).sum(axis=0)
    var_re = (cr ** 2 * er ** 2 + ci ** 2 * ei ** 2).sum(axis=0)
    var_im = (cr ** 2 * ei ** 2 + ci ** 2 * er ** 2).sum(axis=0)
    return re, im, np.sqrt(var_re), np.sqrt(var_im)


def amplitude_series(coef, ival, ierr):
    """Sum with regulator-dependent coefficients (Sec. 2.4): coef [NI, P] holds the Laurent
    terms c_p of each integral's coefficient, and the product of series gives
        A_j = sum_i sum_{p <= j} c_ip I_i,j-p,   var(Re A_j) = sum (Re c_ip)^2 var(I_i,j-p)
    (likewise Im), the orders of an integral counted as independent (the per-order
    propagation of Sec. 2.1.3, Eq. 4, applied term by term).  Real integrals.
    Returns (re, im, err_re, err_im), each of shape [K]."""
    C = np.asarray(coef, dtype=np.complex128)
    ir = np.asarray(ival, dtype=np.float64)
    er = np.asarray(ierr, dtype=np.float64)
    NI, K = ir.shape
    re, im, vre, vim = (np.zeros(K) for _ in range(4))
    for j in range(K):
        for i in range(NI):
            for p in range(min(C.shape[1], j + 1)):
                c = C[i, p]
                re[j] += c.real * ir[i, j - p]
                im[j] += c.imag * ir[i, j - p]
                vre[j] += c.real ** 2 * er[i, j - p] ** 2
                vim[j] += c.imag ** 2 * er[i, j - p] ** 2
    return re, im, np.sqrt(vre), np.sqrt(vim)


def eps_rel(re, im, dre, dim):
    """epsilon_rel = sqrt((dR^2 + dI^2) / (R^2 + I^2)) (Sec. 3.2, timing notes)."""
    return np.sqrt((np.asarray(dre) ** 2 + np.asarray(dim) ** 2) /
                   (np.asarray(re) ** 2 + np.asarray(im) ** 2))


# --------------------------------------------------------------- allocation

def allocate(c2, w, tau, V, alpha: float = 2.0):
    """Lattice sizes minimising T = sum tau_i n_i subject to sum |C_i|^2 w_i / n_i^alpha = V.

    Lagrange solution of Sec. 2.1.3 (Eq. adaptive-solution), read with one consistent unit
    index i (the printed equation mixes the sum and free indices):
        lambda = (1/alpha) [ (1/V) sum_i (|C_i|^2 w_i tau_i^alpha)^(1/(alpha+1)) ]^((alpha+1)/alpha)
        n_i    = (alpha w_i lambda |C_i|^2 / tau_i)^(1/(alpha+1))
    Units with zero |C_i|^2 w_i get n_i = 0.  Returns (n [real], lambda).
    """
    c2 = np.asarray(c2, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    s = np.sum((c2 * w * tau ** alpha) ** (1.0 / (alpha + 1.0)))
    lam = (1.0 / alpha) * (s / V) ** ((alpha + 1.0) / alpha)
    n = (alpha * w * lam * c2 / tau) ** (1.0 / (alpha + 1.0))
    return n, lam


# ------------------------------------------------------------ adaptive sums

def adaptive_amplitude(problem, coef, lattice_n, lattice_a, tau, epsrel, epsabs=0.0,
                       alpha=2.0, n_presample=10000, max_rounds=50, threads=8, trace=None):
    """Adaptive evaluation of weighted sums of integrals, Sec. 2.1.3 (reading: the unit
    is a sector; its coefficient is its integral's; unmet (sum, order) targets are
    processed in order keeping each sector's largest request; sizes never shrink and
    are rounded up to the table of available lattices).

    coef: complex [n_sums, n_integrals], or [n_sums, n_integrals, P] Laurent terms of
    regulator-dependent coefficients (Sec. 2.4; see amplitude_series: a target (t, j)
    weighs sector s by sum_p |c_p|^2 w_s,j-p).  lattice_n: ascending sizes; lattice_a:
    [L, 8] Korobov parameter per size and dimension (column d-1).  tau: cost per
    evaluation of each sector: an array [S], or [R, S] with row r the costs the
    allocation after round r + 1 uses (the last row for later rounds).  Returns
    (value [T, K] complex, error [T, K] complex (err_re + 1j err_im), n_final [S], rounds,
    converged).  trace: if a list, one record per round is appended, holding what the
    round measured and decided: n (lattice sizes integrated), mean and err [S, K],
    tau [S], and per unmet target (t, k) its variance bound V and the closed-form sizes
    n_opt [S] before the never-shrink maximum and the ladder ceiling (0 where a sector
    does not contribute).
    """
    C = np.asarray(coef, dtype=np.complex128)
    if C.ndim == 1:
        C = C[None, :]
    if C.ndim == 2:
        C = C[:, :, None]
    T, NI, P = C.shape
    S = len(problem.sectors)
    K = problem.K
    lad = [int(v) for v in lattice_n]
    la = np.asarray(lattice_a, dtype=np.uint64).reshape(len(lad), 8)
    tau_rows = np.atleast_2d(np.asarray(tau, dtype=np.float64))

    def ceil_index(x):
        for l, v in enumerate(lad):
            if v >= x:
                return l
        return len(lad) - 1

    lidx = [ceil_index(max(n_presample, 2))] * S
    Q = [None] * S
    active = [True] * S
    rounds = 0
    converged = False
    while True:
        todo = [s for s in range(S) if active[s]]

        def run(s):
            sec = problem.sectors[s]
            n = lad[lidx[s]]
            a = int(la[lidx[s], sec.d - 1])
            Q[s] = sector_sums(sec, problem.shifts[s], n=n, a=a)[0]

        if threads > 1:
            with ThreadPoolExecutor(max_workers=threads) as ex:
                list(ex.map(run, todo))
        else:
            for s in todo:
                run(s)
        rounds += 1
        mean = np.zeros((S, K))
        err = np.zeros((S, K))
        for s in range(S):
            mean[s], err[s] = estimate(Q[s])
        ival, ierr = integral_values(problem, list(mean), list(err))
        vals = np.zeros((T, K), dtype=np.complex128)
        errs = np.zeros((T, K), dtype=np.complex128)
        unmet = []
        for t in range(T):
            re, im, dre, dim_ = amplitude_series(C[t], ival, ierr)
            vals[t] = re + 1j * im
            errs[t] = dre + 1j * dim_
            for k in range(K):
                mag2 = re[k] ** 2 + im[k] ** 2
                var = dre[k] ** 2 + dim_[k] ** 2
                eps = math.sqrt(var / mag2) if mag2 > 0 else (math.inf if var > 0 else 0.0)
                if not (eps <= epsrel or math.sqrt(var) <= epsabs):
                    unmet.append((t, k, mag2))
        tau = tau_rows[min(rounds - 1, tau_rows.shape[0] - 1)]
        n_cur = np.array([lad[lidx[s]] for s in range(S)], dtype=np.float64)
        rec = None
        if trace is not None:
            rec = {"n": n_cur.copy(), "mean": mean.copy(), "err": err.copy(),
                   "tau": tau.copy(), "targets": []}
            trace.append(rec)
        if not unmet:
            converged = True
            break
        if rounds > max_rounds:
            break
        want = n_cur.copy()
        for t, k, mag2 in unmet:
            V = max(epsrel ** 2 * mag2, epsabs ** 2)
            if not V > 0:
                continue
            # |C|^2 w_s summed over the coefficient terms that reach order k
            cw = np.zeros(S)
            for s in range(S):
                ci = C[t, problem.sectors[s].integral]
                cw[s] = sum(abs(ci[p]) ** 2 * err[s, k - p] ** 2
                            for p in range(min(P, k + 1))) * n_cur[s] ** alpha
            use = cw > 0
            if not use.any():
                continue
            n_opt, _ = allocate(np.ones(int(use.sum())), cw[use], tau[use], V, alpha)
            want[use] = np.maximum(want[use], n_opt)
            if rec is not None:
                full = np.zeros(S)
                full[use] = n_opt
                rec["targets"].append({"t": t, "k": k, "V": V, "n_opt": full})
        new = [max(lidx[s], ceil_index(want[s])) for s in range(S)]
        active = [new[s] != lidx[s] for s in range(S)]
        lidx = new
        if not any(active):
            break
    n_final = np.array([lad[l] for l in lidx], dtype=np.uint64)
    return vals, errs, n_final, rounds, converged
