"""Seeded synthetic inputs for randomized rank-1 lattice QMC over sector integrands.

This module holds random draws only: sector shapes, monomial exponents and
coefficients of the U and F polynomials, lattice sizes (primes), candidate
Korobov parameters, random shifts, kinematic invariants and amplitude
coefficients.  It evaluates no integrand, lattice point, transform, sum,
error estimate or lattice-size allocation: both the CPU oracle and the HIP
library consume exactly these arrays and do the arithmetic of the method on
their own.

The shapes follow the integrands the paper targets (sector-decomposed
Feynman-parameter integrals, paper Sec. 2.1 and Sec. 3): after the delta
constraint an L-loop graph with N propagators has d = N - 1 Feynman
parameters, U has degree L and F degree L + 1 (inhomogeneous, constant term
present, Euclidean kinematics so F > 0 on the unit cube), and the
epsilon-expansion of U^a F^(b + c*eps) produces powers of log F per order.
The paper's own example integrands are generated code that is not available
here; these seeded stand-ins reproduce their dimensions, degrees, term counts
and lattice sizes.

Integrand convention (shared by both implementations):

    f_k(x) = x^p * U(x)^a * F(x)^b * sum_m logc[k, m] * (log F(x))^m

for order index k = 0..K-1 (epsilon power ``order_lo + k``), with
p_j = x_pow2[j] / 2, b = f_pow2 / 2 (half-integers allowed) and integer a.
"""

from __future__ import annotations

import dataclasses
import math
from fractions import Fraction
from typing import List, Optional

import numpy as np

TRANSFORMS = ("none", "baker", "korobov1", "korobov2", "korobov3", "korobov4",
              "korobov5", "korobov6")


@dataclasses.dataclass
class Sector:
    d: int
    u_exp: np.ndarray      # uint8 [n_u, d]
    u_coef: np.ndarray     # float64 [n_u]
    f_exp: np.ndarray      # uint8 [n_f, d]
    f_coef: np.ndarray     # float64 [n_f]
    x_pow2: np.ndarray     # int32 [d], twice the exponent of x_j
    u_pow: int             # integer exponent of U
    f_pow2: int            # twice the exponent of F
    logc: np.ndarray       # float64 [K, M+1], coefficient of (log F)^m in order k
    n: int                 # lattice size
    a: int                 # Korobov parameter: generating vector (1, a, a^2, ...) mod n
    transform: str = "korobov3"
    integral: int = 0      # parent integral index (a sum of sectors)
    a_candidates: Optional[np.ndarray] = None  # uint64, random candidates for a
    deform_lambda: float = 0.0  # > 0: integrate on the deformed contour (F - i0), complex

    @property
    def K(self) -> int:
        return int(self.logc.shape[0])

    @property
    def M(self) -> int:
        return int(self.logc.shape[1]) - 1


@dataclasses.dataclass
class Problem:
    sectors: List[Sector]
    order_lo: int                 # epsilon power of order index 0
    m: int                        # number of random shifts
    shifts: List[np.ndarray]      # per sector, float64 [m, d] in [0, 1)
    n_integrals: int = 1
    amp_coef: Optional[np.ndarray] = None   # complex128 [n_integrals]: A = sum_i C_i I_i
    name: str = ""
    seed: int = 0

    @property
    def K(self) -> int:
        return self.sectors[0].K

    @property
    def M(self) -> int:
        return max(s.M for s in self.sectors)

    def evals(self) -> int:
        return int(sum(s.n for s in self.sectors)) * self.m


# --------------------------------------------------------------------------
# small helpers: primes (input sizes) and random draws
# --------------------------------------------------------------------------

def _is_prime(n: int) -> bool:
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if n % p == 0:
            return n == p
    dd, s = n - 1, 0
    while dd % 2 == 0:
        dd //= 2
        s += 1
    for a in small:  # deterministic for n < 3.3e24
        x = pow(a, dd, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def next_prime(n: int) -> int:
    """Smallest prime >= n (used to draw prime lattice sizes)."""
    n = max(2, int(n))
    while not _is_prime(n):
        n += 1
    return n


def uniform_shifts(rng: np.random.Generator, m: int, d: int) -> np.ndarray:
    """m shift vectors in [0,1)^d, each coordinate an exact multiple of 2^-53."""
    k = rng.integers(0, 1 << 53, size=(m, d), dtype=np.int64)
    return k.astype(np.float64) * (2.0 ** -53)


def _monomials(d: int, deg_lo: int, deg_hi: int) -> List[tuple]:
    out = []

    def rec(prefix, left, pos):
        if pos == d:
            if deg_lo <= sum(prefix) <= deg_hi:
                out.append(tuple(prefix))
            return
        for e in range(left, -1, -1):
            rec(prefix + [e], left - e, pos + 1)

    rec([], deg_hi, 0)
    out.sort(key=lambda t: (sum(t), tuple(-e for e in t)))
    return out


def random_polynomial(rng: np.random.Generator, d: int, count: int, deg: int,
                      lo: float = 0.1, hi: float = 1.0):
    """Constant term plus (count-1) distinct monomials of total degree 1..deg.

    Coefficients are drawn from U(lo, hi).  The count is capped at the number
    of available monomials.
    """
    pool = _monomials(d, 1, deg)
    k = min(count - 1, len(pool))
    pick = rng.choice(len(pool), size=k, replace=False)
    exps = [tuple([0] * d)] + [pool[i] for i in sorted(pick)]
    coef = rng.uniform(lo, hi, size=len(exps))
    return np.array(exps, dtype=np.uint8).reshape(len(exps), d), coef.astype(np.float64)


def _korobov_candidates(rng: np.random.Generator, n: int, count: int) -> np.ndarray:
    if n < 4:
        return np.ones(count, dtype=np.uint64)
    return rng.integers(2, n - 1, size=count, dtype=np.int64).astype(np.uint64)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def one_loop_sector(seed: int = 0, n: int = 65521, m: int = 16, a: Optional[int] = None,
                    transform: str = "korobov3") -> Problem:
    """Single one-loop-like sector: d = 3, U = 1 + x1 + x2, F = constant + 5 monomials of
    degree <= 2 with coefficients U(0.1, 1); integrand x1^(1/2) U^-1 F^(-1-eps) expanded to
    two orders: x1^(1/2)/(U F) and -x1^(1/2) log(F)/(U F).  Korobov lattice of size n,
    16 shifts."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    d = 3
    u_exp = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], dtype=np.uint8)
    u_coef = np.ones(3)
    pool = _monomials(d, 1, 2)                       # the 9 non-constant monomials
    pick = sorted(rng.choice(len(pool), size=5, replace=False))
    f_exp = np.array([[0, 0, 0]] + [pool[i] for i in pick], dtype=np.uint8)
    f_coef = rng.uniform(0.1, 1.0, size=6)
    cands = _korobov_candidates(rng, n, 64)
    shifts = uniform_shifts(rng, m, d)
    sec = Sector(d=d, u_exp=u_exp, u_coef=u_coef, f_exp=f_exp, f_coef=f_coef,
                 x_pow2=np.array([1, 0, 0], dtype=np.int32), u_pow=-1, f_pow2=-2,
                 logc=np.array([[1.0, 0.0], [0.0, -1.0]]), n=n,
                 a=int(cands[0]) if a is None else int(a), transform=transform,
                 a_candidates=cands)
    return Problem(sectors=[sec], order_lo=0, m=m, shifts=[shifts], name="one_loop_sector",
                   seed=seed)


TWO_LOOP_LOGC = np.array([[1.0, 0.0, 0.0],     # eps^-2 :  U F^-3
                          [0.0, -2.0, 0.0],    # eps^-1 :  U F^-3 (-2 log F)
                          [0.0, 0.0, 2.0]])    # eps^0  :  U F^-3 (-2 log F)^2 / 2


def _two_loop_sector(rng, d, n, integral, transform="korobov3", n_cand=64):
    nu = int(rng.integers(4, 9))
    nf = int(rng.integers(10, 31))
    u_exp, u_coef = random_polynomial(rng, d, nu, 2)
    f_exp, f_coef = random_polynomial(rng, d, nf, 3)
    cands = _korobov_candidates(rng, n, n_cand)
    return Sector(d=d, u_exp=u_exp, u_coef=u_coef, f_exp=f_exp, f_coef=f_coef,
                  x_pow2=np.zeros(d, dtype=np.int32), u_pow=1, f_pow2=-6,
                  logc=TWO_LOOP_LOGC.copy(), n=n, a=int(cands[0]), transform=transform,
                  integral=integral, a_candidates=cands)


def two_loop_integral(seed: int = 0, n_sectors: int = 40, d_lo: int = 4, d_hi: int = 6,
                      log10n_lo: float = 5.0, log10n_hi: float = 7.0, m: int = 32,
                      n_scale: float = 1.0) -> Problem:
    """Two-loop-like integral: n_sectors sectors, d uniform in [d_lo, d_hi], U with 4-8
    monomials (constant + degree 1..2), F with 10-30 monomials (constant + degree 1..3),
    coefficients U(0.1, 1); integrand eps^-2 U F^(-3-2 eps) expanded to orders -2..0
    (log^m F, m <= 2).  Per-sector prime lattice sizes log-uniform in
    [10^log10n_lo, 10^log10n_hi] (times n_scale, for reduced test sizes), m shifts."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 2])))
    secs, shifts = [], []
    for _ in range(n_sectors):
        d = int(rng.integers(d_lo, d_hi + 1))
        n = next_prime(int(math.ceil(n_scale * 10.0 ** rng.uniform(log10n_lo, log10n_hi))))
        secs.append(_two_loop_sector(rng, d, n, 0))
        shifts.append(uniform_shifts(rng, m, d))
    return Problem(sectors=secs, order_lo=-2, m=m, shifts=shifts, name="two_loop_integral",
                   seed=seed)


def _physical_sector(rng, d, n, integral, s1, s2, lam, shapes=None):
    """Sector of a physical-region scan point: U as the two-loop sectors; F has the
    two-loop monomial structure with coefficients alpha_t - beta_t s1 - gamma_t s2,
    alpha, beta, gamma ~ U(0.1, 1), so F changes sign on the cube.  `shapes` reuses
    (u_exp, u_coef, f_exp, alpha, beta, gamma, a) of a base sector across points."""
    if shapes is None:
        nu = int(rng.integers(4, 9))
        nf = int(rng.integers(10, 31))
        u_exp, u_coef = random_polynomial(rng, d, nu, 2)
        f_exp, _ = random_polynomial(rng, d, nf, 3)
        al, be, ga = (rng.uniform(0.1, 1.0, size=len(f_exp)) for _ in range(3))
        a = int(_korobov_candidates(rng, n, 1)[0])
        shapes = (u_exp, u_coef, f_exp, al, be, ga, a)
    u_exp, u_coef, f_exp, al, be, ga, a = shapes
    f_coef = al - be * s1 - ga * s2
    sec = Sector(d=d, u_exp=u_exp, u_coef=u_coef, f_exp=f_exp, f_coef=f_coef,
                 x_pow2=np.zeros(d, dtype=np.int32), u_pow=1, f_pow2=-6,
                 logc=TWO_LOOP_LOGC.copy(), n=n, a=a, transform="korobov3",
                 integral=integral, deform_lambda=lam)
    return sec, shapes


def physical_scan(seed: int = 0, n_points: int = 1000, n_sectors: int = 200, d_lo: int = 3,
                  d_hi: int = 8, n: int = 65521, m: int = 16, lam: float = 0.5) -> Problem:
    """Physical-region scan: n_points kinematic points (s1, s2 ~ U(1, 10)) times the same
    n_sectors base sectors (d uniform in [d_lo, d_hi]); sector (p, b) belongs to integral
    p.  Integrand eps^-2 U F^(-3-2 eps) to orders -2..0 as the two-loop sectors, on the
    deformed contour with initial parameter lam; lattice size n, m shifts."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 5])))
    base = []
    for _ in range(n_sectors):
        d = int(rng.integers(d_lo, d_hi + 1))
        base.append((d, None))
    kin = rng.uniform(1.0, 10.0, size=(n_points, 2))
    secs, shifts = [], []
    for p in range(n_points):
        for b in range(n_sectors):
            d, shapes = base[b]
            sec, shapes = _physical_sector(rng, d, n, p, kin[p, 0], kin[p, 1], lam, shapes)
            base[b] = (d, shapes)
            secs.append(sec)
            shifts.append(uniform_shifts(rng, m, d))
    prob = Problem(sectors=secs, order_lo=-2, m=m, shifts=shifts, n_integrals=n_points,
                   name="physical_scan", seed=seed)
    prob.kinematics = kin
    return prob


def _rational_in(rng, nvars=3, lo=-9, hi=9, nonneg=False):
    mons = _monomials(nvars, 0, 2)
    if nonneg:
        c = rng.integers(0, 10, size=len(mons))
    else:
        c = rng.integers(lo, hi + 1, size=len(mons))
    return mons, [int(v) for v in c]


def amplitude(seed: int = 0, n_integrals: int = 20, n_sectors: int = 500, d_lo: int = 3,
              d_hi: int = 7, m: int = 32, n0: int = 10007) -> Problem:
    """Synthetic amplitude A = sum_i c_i I_i over n_integrals two-loop-like integrals
    totalling n_sectors sectors (each integral gets at least one sector, the rest are
    assigned uniformly at random, so sizes are uneven), d uniform in [d_lo, d_hi].  The
    coefficients c_i = P_i(s)/Q_i(s) are rational functions of three kinematic invariants
    s_j in [1, 10] (P_i: integer coefficients in [-9, 9], Q_i: 1 + non-negative integer
    coefficients in [0, 9], both on monomials of degree <= 2), evaluated exactly in
    rationals and rounded once to float64.  All sectors start at lattice size n0."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 3])))
    owner = list(range(n_integrals)) + [int(v) for v in
                                         rng.integers(0, n_integrals, size=n_sectors - n_integrals)]
    secs, shifts = [], []
    for s in range(n_sectors):
        d = int(rng.integers(d_lo, d_hi + 1))
        secs.append(_two_loop_sector(rng, d, n0, owner[s], n_cand=16))
        shifts.append(uniform_shifts(rng, m, d))
    inv = [Fraction(int(rng.integers(1000, 10001)), 1000) for _ in range(3)]
    coefs = []
    for _ in range(n_integrals):
        mons, pc = _rational_in(rng)
        _, qc = _rational_in(rng, nonneg=True)
        num = Fraction(0)
        den = Fraction(1)
        for e, a, b in zip(mons, pc, qc):
            mv = inv[0] ** e[0] * inv[1] ** e[1] * inv[2] ** e[2]
            num += a * mv
            den += b * mv
        if num == 0:
            num = Fraction(1)
        coefs.append(float(num / den))
    return Problem(sectors=secs, order_lo=-2, m=m, shifts=shifts, n_integrals=n_integrals,
                   amp_coef=np.array(coefs, dtype=np.complex128), name="amplitude", seed=seed)


def coefficient_expressions(seed: int = 0, n_integrals: int = 20):
    """Coefficient strings of an amplitude in the form reduction programs produce them:
    c_i = P_i(s)/Q_i(s) * R_i(d) with three kinematic invariants s1..s3 (decimals in
    [1, 10]), P_i with integer coefficients in [-9, 9] and Q_i = 1 + non-negative integer
    coefficients on monomials of degree <= 2, and R_i(d) a rational factor in the
    space-time dimension d = 4 - 2 eps (some with a pole in eps).  Returns (expressions
    [n_integrals], symbol values {name: value string})."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 31])))
    mons = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (0, 1, 1),
            (0, 0, 2)]
    d_factors = ["1", "(d-2)/(d-3)", "1/(d-4)", "(3*d-10)/(2*(d-4))", "(d-4)/(d-6)",
                 "(d-1)^2/((d-3)*(d-5))"]

    def mono(e):
        f = [f"s{j + 1}^{p}" if p > 1 else f"s{j + 1}" for j, p in enumerate(e) if p]
        return "*".join(f) if f else "1"

    exprs = []
    for _ in range(n_integrals):
        k = int(rng.integers(2, 6))
        pick = rng.choice(len(mons), size=k, replace=False)
        num = " + ".join(f"({int(rng.integers(-9, 10))})*{mono(mons[i])}" for i in pick)
        den = "1 + " + " + ".join(f"{int(rng.integers(0, 10))}*{mono(mons[i])}"
                                  for i in rng.choice(len(mons), size=3, replace=False))
        exprs.append(f"({num})/({den})*{d_factors[int(rng.integers(0, len(d_factors)))]}")
    symbols = {f"s{j + 1}": f"{int(rng.integers(1000, 10001)) / 1000:.3f}" for j in range(3)}
    symbols["d"] = "4-2*eps"
    return exprs, symbols


def custom_sector(d, u_terms, f_terms, x_pow2=None, u_pow=0, f_pow2=0, logc=((1.0,),),
                  n=1009, a=1, transform="none", integral=0, deform_lambda=0.0) -> Sector:
    """A hand-specified sector: u_terms / f_terms are lists of (coef, exponent tuple)."""
    def poly(terms):
        if not terms:
            return np.zeros((0, d), dtype=np.uint8), np.zeros(0)
        e = np.array([t[1] for t in terms], dtype=np.uint8).reshape(len(terms), d)
        c = np.array([t[0] for t in terms], dtype=np.float64)
        return e, c
    ue, uc = poly(u_terms)
    fe, fc = poly(f_terms)
    return Sector(d=d, u_exp=ue, u_coef=uc, f_exp=fe, f_coef=fc,
                  x_pow2=np.zeros(d, np.int32) if x_pow2 is None else np.asarray(x_pow2, np.int32),
                  u_pow=u_pow, f_pow2=f_pow2, logc=np.asarray(logc, dtype=np.float64),
                  n=n, a=a, transform=transform, integral=integral,
                  deform_lambda=float(deform_lambda))


def single_problem(sector: Sector, m: int = 8, seed: int = 0, order_lo: int = 0) -> Problem:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 9])))
    return Problem(sectors=[sector], order_lo=order_lo, m=m,
                   shifts=[uniform_shifts(rng, m, sector.d)], seed=seed)


def median_candidates(rng, n: int, d: int, r: int) -> np.ndarray:
    """r random generating vectors [r, d] with every component uniform in
    U_n = {1 <= z <= n - 1 : gcd(z, n) = 1} (rejection sampling)."""
    out = np.empty((r, d), dtype=np.uint64)
    for c in range(r):
        for j in range(d):
            while True:
                z = int(rng.integers(1, n))
                if math.gcd(z, n) == 1:
                    out[c, j] = z
                    break
    return out


def lattice_ladder(n_min: int = 10007, n_max: int = 2 ** 31 - 1, ratio: float = 1.5,
                   n_cand: int = 8, seed: int = 0):
    """Table of available lattice sizes (primes near n_min * ratio^l, up to n_max) with
    n_cand random Korobov-parameter candidates per size and dimension (the role of a
    precomputed generating-vector table).  Returns (sizes uint64 [L],
    candidates uint64 [L, QMC_MAX_DIM = 8, n_cand])."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11])))
    sizes = []
    v = float(n_min)
    while True:
        p = next_prime(int(math.ceil(v)))
        if p > n_max:
            break
        if not sizes or p > sizes[-1]:
            sizes.append(p)
        v *= ratio
    cands = np.stack([np.stack([_korobov_candidates(rng, n, n_cand) for _ in range(8)])
                      for n in sizes])
    return np.array(sizes, dtype=np.uint64), cands
