"""Pins of the CPU oracle against mathematics: closed forms, identities, brute force.

None of these tests retypes an oracle formula.  Each one compares the oracle with a
result fixed independently of it (a closed-form integral, a character-sum identity,
a textbook statistic, a brute-force minimum, a truncated series), chosen so that a
plausible slip in the oracle (dropped term, wrong sign or index, transposed exponent,
missing shift, wrong modulus) fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy import integrate as sint
from scipy import optimize

import oracle
import workloads as W


# ----------------------------------------------------------------- lattice

@pytest.mark.parametrize("n,a", [(101, 12), (1009, 317), (65521, 17364)])
def test_lattice_columns_are_permutations(n, a):
    z = oracle.korobov_vector(n, a, 4)
    y = oracle.points(n, z, np.zeros(4))
    k = np.rint(y * n).astype(np.int64)
    assert np.array_equal(k[:, 0], np.arange(n))          # z_1 = 1 gives k_1 = i
    for j in range(4):
        assert np.array_equal(np.sort(k[:, j]), np.arange(n))   # gcd(z_j, n) = 1
        # k_j = i z_j mod n, brute force in Python integers
        assert all(int(k[i, j]) == (i * int(z[j])) % n for i in range(0, n, max(1, n // 97)))


def test_lattice_quotient_is_ieee_and_shift_wraps_exactly():
    n, a = 1009, 317
    z = oracle.korobov_vector(n, a, 3)
    delta = np.array([0.75, 0.5 + 2.0 ** -40, 1.0 - 2.0 ** -53])
    y = oracle.points(n, z, delta)
    for i in (0, 1, 500, 1008):
        for j in range(3):
            q = ((i * int(z[j])) % n) / n          # Python float division is IEEE RN
            v = q + delta[j]
            v = v - 1.0 if v >= 1.0 else v
            assert y[i, j] == v
            assert 0.0 <= y[i, j] < 1.0


def _trig_poly(x, terms):
    f = np.zeros(x.shape[0], dtype=np.complex128)
    for h, c in terms:
        f += c * np.exp(2j * np.pi * (x @ np.asarray(h, dtype=np.float64)))
    return f


def test_lattice_rule_exact_on_trig_polynomials():
    # Q_{n,z}(e^{2 pi i h.x}) = e^{2 pi i h.Delta} if h.z = 0 mod n, else 0 (character sum).
    rng = np.random.default_rng(5)
    n, z = 1009, oracle.korobov_vector(1009, 317, 3)
    hs = [(h1, h2, h3) for h1 in range(-3, 4) for h2 in range(-3, 4) for h3 in range(-3, 4)]
    coef = rng.normal(size=len(hs)) + 1j * rng.normal(size=len(hs))
    terms = list(zip(hs, coef))
    delta = rng.random(3)
    q = _trig_poly(oracle.points(n, z, delta), terms).mean()
    pred = sum(c * np.exp(2j * np.pi * np.dot(h, delta)) for h, c in terms
               if (np.dot(h, z.astype(np.int64)) % n) == 0)
    const = dict(terms)[(0, 0, 0)]
    assert abs(pred - const) < 1e-15          # no small nonzero h is aliased for this z
    assert abs(q - pred) < 1e-12


def test_lattice_rule_aliases_predicted_dual_vectors():
    # Small lattice where short dual vectors exist: n = 7, z = (1, 2, 4).
    n, z = 7, oracle.korobov_vector(7, 2, 3)
    assert list(z) == [1, 2, 4]
    terms = [((0, 0, 0), 0.3), ((-2, 1, 0), 1.0 + 0.5j), ((1, 1, 1), 0.7), ((1, 0, 0), 2.0),
             ((0, -2, 1), -0.4j)]
    rng = np.random.default_rng(1)
    for _ in range(5):
        delta = rng.random(3)
        q = _trig_poly(oracle.points(n, z, delta), terms).mean()
        dual = [(h, c) for h, c in terms if np.dot(h, [1, 2, 4]) % 7 == 0]
        assert {h for h, _ in dual} == {(0, 0, 0), (-2, 1, 0), (1, 1, 1), (0, -2, 1)}
        pred = sum(c * np.exp(2j * np.pi * np.dot(h, delta)) for h, c in dual)
        assert abs(q - pred) < 1e-13


# --------------------------------------------------------------- transforms

@pytest.mark.parametrize("kind,r", [("korobov1", 1), ("korobov2", 2), ("korobov3", 3),
                                    ("korobov4", 4), ("korobov6", 6)])
def test_korobov_transform_properties(kind, r):
    y = np.linspace(0.0, 1.0, 1001)
    x, w = oracle.transform(kind, y)
    assert x[0] == 0.0 and abs(x[-1] - 1.0) < 1e-14
    x_rev, _ = oracle.transform(kind, 1.0 - y)
    assert np.max(np.abs(x_rev - (1.0 - x))) < 1e-13            # phi(1-y) = 1 - phi(y)
    assert np.all(np.diff(x) >= 0.0)
    # w = phi' (central differences) and w = (2r+1)!/(r!)^2 (y(1-y))^r
    h = 1e-6
    yy = np.linspace(0.01, 0.99, 97)
    xp, _ = oracle.transform(kind, yy + h)
    xm, _ = oracle.transform(kind, yy - h)
    _, ww = oracle.transform(kind, yy)
    assert np.max(np.abs((xp - xm) / (2 * h) - ww)) < 1e-7
    cst = math.factorial(2 * r + 1) / math.factorial(r) ** 2
    assert np.max(np.abs(ww - cst * (yy * (1 - yy)) ** r)) < 1e-12
    # int_0^1 w = 1 and int f(phi) phi' = int f for f = x^2 (Gauss-Legendre, exact here)
    t, gw = np.polynomial.legendre.leggauss(40)
    yg = 0.5 * (t + 1.0)
    xg, wg = oracle.transform(kind, yg)
    assert abs(0.5 * np.dot(gw, wg) - 1.0) < 1e-14
    assert abs(0.5 * np.dot(gw, wg * xg ** 2) - 1.0 / 3.0) < 1e-14


def test_korobov3_is_the_degree7_polynomial():
    y = np.linspace(0, 1, 257)
    x, w = oracle.transform("korobov3", y)
    # the regularized incomplete beta I_y(4, 4), written in monomials
    assert np.max(np.abs(x - y ** 4 * (35 - 84 * y + 70 * y ** 2 - 20 * y ** 3))) < 1e-13
    assert np.max(np.abs(w - 140 * y ** 3 * (1 - y) ** 3)) < 1e-13


def test_baker_is_tent_map():
    y = np.array([0.0, 0.25, 0.5, 0.75, 0.999])
    x, w = oracle.transform("baker", y)
    assert np.allclose(x, [0.0, 0.5, 1.0, 0.5, 0.002], atol=1e-15)
    assert np.all(w == 1.0)


# ------------------------------------------------ integrand via closed forms

def _integrate(sec, m=8, seed=3, threads=4):
    prob = W.single_problem(sec, m=m, seed=seed)
    Q, _ = oracle.sector_sums(sec, prob.shifts[0], threads=threads)
    return oracle.estimate(Q)


def test_bubble_log_moments():
    """One-loop massless bubble: int_0^1 [x(1-x)]^(-eps) dx = Gamma(1-eps)^2/Gamma(2-2eps)
    = 1 + 2 eps + (4 - pi^2/6) eps^2 + O(eps^3).  By symmetry x -> t/2 on [0, 1/2]:
    F = t/2 - t^2/4, and the eps^m coefficient is int (-log F)^m / m!."""
    sec = W.custom_sector(1, [], [(0.5, (1,)), (-0.25, (2,))],
                          logc=[[1, 0, 0], [0, -1, 0], [0, 0, 0.5]], n=100003, a=1,
                          transform="korobov3")
    mean, err = _integrate(sec)
    exact = np.array([1.0, 2.0, 4.0 - math.pi ** 2 / 6.0])
    assert np.all(np.abs(mean - exact) < 1e-9 + 5 * err)
    assert np.all(err < 1e-9)


@pytest.mark.parametrize("case", ["F^-3", "U F^-3", "x^1/2 F^-1", "F^-1/2", "logF/F",
                                  "U^-1 F^-2"])
def test_closed_form_integrals(case):
    two_d = False
    if case == "F^-3":       # int (1+x)^-3 = 3/8
        sec = W.custom_sector(1, [], [(1, (0,)), (1, (1,))], f_pow2=-6)
        exact = 3 / 8
    elif case == "U F^-3":   # int (1+2x)(1+x)^-3 = 5/8
        sec = W.custom_sector(1, [(1, (0,)), (2, (1,))], [(1, (0,)), (1, (1,))], u_pow=1,
                              f_pow2=-6)
        exact = 5 / 8
    elif case == "x^1/2 F^-1":   # int sqrt(x)/(1+x) = 2 - pi/2
        sec = W.custom_sector(1, [], [(1, (0,)), (1, (1,))], x_pow2=[1], f_pow2=-2)
        exact = 2 - math.pi / 2
    elif case == "F^-1/2":   # int (1+x)^-1/2 = 2(sqrt 2 - 1)
        sec = W.custom_sector(1, [], [(1, (0,)), (1, (1,))], f_pow2=-1)
        exact = 2 * (math.sqrt(2) - 1)
    elif case == "logF/F":   # int log(1+x)/(1+x) = log^2(2)/2
        sec = W.custom_sector(1, [], [(1, (0,)), (1, (1,))], f_pow2=-2, logc=[[0, 1]])
        exact = math.log(2) ** 2 / 2
    else:                    # int int (1+x1)^-1 (1+x2)^-2 = log(2)/2
        two_d = True
        sec = W.custom_sector(2, [(1, (0, 0)), (1, (1, 0))], [(1, (0, 0)), (1, (0, 1))],
                              u_pow=-1, f_pow2=-4)
        exact = math.log(2) / 2
    sec.n, sec.a, sec.transform = (10007, 3051, "korobov3") if two_d else (10007, 1, "korobov3")
    mean, err = _integrate(sec)
    assert abs(mean[0] - exact) < 1e-9 + 5 * err[0]
    assert err[0] < 1e-7


def box6_problem(S, T, n=65521, a=17364, m=8, seed=7):
    """The one-loop massless box in D = 6 (finite) as a sum of sector integrals.

    With Feynman parameters x_1..x_4 and Euclidean invariants S = -s > 0, T = -t > 0, the
    box's parameter integral is J = int dx delta(1 - sum x) U^-2 F^-1, U = x1 + x2 + x3 + x4,
    F = S x1 x3 + T x2 x4 (the D = 6 exponents N - D = -2 and -(N - D/2) = -1).  Its known
    closed form is J(S, T) = (log^2(S/T) + pi^2) / (2 (S + T)).

    Sector decomposition, derived by hand: the primary sector x1 = 1 (the others in [0,1]:
    t2, t3, t4) has U = 1 + t2 + t3 + t4 and F = S t3 + T t2 t4, which vanishes on
    {t3 = 0, t2 t4 = 0}.  Splitting (t3, t2) by which is larger and then (u3, t4):
      (a)  t2 = t3 u2:             F = t3 (S + T u2 t4),  Jacobian t3
      (b1) t3 = t2 u3, u3 = t4 v:  F = t2 t4 (S v + T),   Jacobian t2 t4
      (b2) t3 = t2 u3, t4 = u3 w:  F = t2 u3 (S + T w),   Jacobian t2 u3
    The Jacobian cancels F's monomial factor in each case, leaving U^-2 G^-1 with a
    positive G: smooth on the cube.  x3 = 1 gives the same three (F is symmetric under
    x1 <-> x3), x2 = 1 and x4 = 1 the same with S <-> T: 12 sectors, one integral."""
    def three(S_, T_):
        return [
            # (a) variables (u2, t3, t4): U = 1 + u2 t3 + t3 + t4, G = S + T u2 t4
            ([(1.0, (0, 0, 0)), (1.0, (1, 1, 0)), (1.0, (0, 1, 0)), (1.0, (0, 0, 1))],
             [(S_, (0, 0, 0)), (T_, (1, 0, 1))]),
            # (b1) variables (t2, v, t4): U = 1 + t2 + t2 v t4 + t4, G = S v + T
            ([(1.0, (0, 0, 0)), (1.0, (1, 0, 0)), (1.0, (1, 1, 1)), (1.0, (0, 0, 1))],
             [(T_, (0, 0, 0)), (S_, (0, 1, 0))]),
            # (b2) variables (t2, u3, w): U = 1 + t2 + t2 u3 + u3 w, G = S + T w
            ([(1.0, (0, 0, 0)), (1.0, (1, 0, 0)), (1.0, (1, 1, 0)), (1.0, (0, 1, 1))],
             [(S_, (0, 0, 0)), (T_, (0, 0, 1))]),
        ]
    polys = three(S, T) * 2 + three(T, S) * 2
    secs = [W.custom_sector(3, u, f, u_pow=-2, f_pow2=-2, n=n, a=a, transform="korobov3")
            for u, f in polys]
    rng = np.random.default_rng(seed)
    shifts = [W.uniform_shifts(rng, m, 3) for _ in secs]
    prob = W.Problem(sectors=secs, order_lo=0, m=m, shifts=shifts, n_integrals=1)
    exact = (math.log(S / T) ** 2 + math.pi ** 2) / (2.0 * (S + T))
    return prob, exact


@pytest.mark.parametrize("S,T", [(1.0, 1.0), (3.7, 1.3), (0.2, 6.0)])
def test_massless_box_six_dimensions_closed_form(S, T):
    """Twelve sector integrals of the hand-decomposed D = 6 massless box sum to the closed
    form: pins multi-dimensional sectors (d = 3, monomials of total degree up to 3, negative
    powers of U and F) added into one integral with their variances."""
    prob, exact = box6_problem(S, T)
    means, errs = [], []
    for s, sec in enumerate(prob.sectors):
        Q, _ = oracle.sector_sums(sec, prob.shifts[s], threads=8)
        mu, e = oracle.estimate(Q)
        means.append(mu)
        errs.append(e)
    val, err = oracle.integral_values(prob, means, errs)
    assert err[0, 0] < 1e-9 * exact
    assert abs(val[0, 0] - exact) < 5 * err[0, 0] + 1e-12 * exact, (val[0, 0], exact, err[0, 0])


def test_mixed_monomial_exponents_not_transposed():
    """F = 1 + x1^2 x2.  int int 1/F = pi/2 - log 2 exactly; with the prefactor sqrt(x1) the
    inner x2-integral is log(1+x1^2)/x1^2, leaving a 1-D integral done by adaptive quadrature.
    Transposing the exponent (x1 x2^2) changes the second value."""
    f_terms = [(1, (0, 0)), (1, (2, 1))]
    sec = W.custom_sector(2, [], f_terms, f_pow2=-2, n=100003, a=33647, transform="korobov3")
    mean, err = _integrate(sec)
    assert abs(mean[0] - (math.pi / 2 - math.log(2))) < 1e-9 + 5 * err[0]
    sec2 = W.custom_sector(2, [], f_terms, x_pow2=[1, 0], f_pow2=-2, n=100003, a=33647,
                           transform="korobov3")
    mean2, err2 = _integrate(sec2)
    ref, _ = sint.quad(lambda x: math.sqrt(x) * math.log1p(x * x) / (x * x), 0, 1,
                       epsabs=1e-14, epsrel=1e-14)
    ref_t, _ = sint.quad(lambda x: math.sqrt(x) * math.log1p(x) / x, 0, 1, epsabs=1e-14,
                         epsrel=1e-14)   # int int sqrt(x1) / (1 + x1 x2^2) would be this
    assert abs(mean2[0] - ref) < 1e-8 + 5 * err2[0]
    assert abs(ref - ref_t) > 1e-2


def _gauss_3d_one_loop(prob, nodes=64):
    """Tensor Gauss-Legendre of the one-loop sector, with x1 = t^2 removing the sqrt."""
    sec = prob.sectors[0]
    t, w = np.polynomial.legendre.leggauss(nodes)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    T1, T2, T3 = np.meshgrid(t, t, t, indexing="ij")
    x = np.stack([T1.ravel() ** 2, T2.ravel(), T3.ravel()], axis=1)
    jac = (2 * T1.ravel())
    ww = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel()
    f = oracle.integrand(sec, x)
    return (ww[:, None] * jac[:, None] * f).sum(axis=0)


def test_one_loop_sector_matches_gauss_legendre():
    prob = W.one_loop_sector(seed=0)
    g64 = _gauss_3d_one_loop(prob, 64)
    g96 = _gauss_3d_one_loop(prob, 96)
    assert np.all(np.abs(g64 - g96) < 1e-13 * np.abs(g96))
    Q, _ = oracle.sector_sums(prob.sectors[0], prob.shifts[0], threads=8)
    mean, err = oracle.estimate(Q)
    assert np.all(np.abs(mean - g96) < 5 * err + 1e-12)
    assert np.all(err < 1e-6 * np.abs(g96))


def test_one_loop_sector_in_one_and_two_dimensions_matches_gauss():
    """1-D and 2-D reductions of the one-loop form (x1^(1/2) U^-1 F^-1, -...log F)."""
    for d in (1, 2):
        fe = [(0.4, (0,) * d), (0.7, (1,) + (0,) * (d - 1)), (0.3, (0,) * (d - 1) + (2,))]
        ue = [(1.0, (0,) * d), (1.0, (1,) + (0,) * (d - 1))]
        sec = W.custom_sector(d, ue, fe, x_pow2=[1] + [0] * (d - 1), u_pow=-1, f_pow2=-2,
                              logc=[[1, 0], [0, -1]], n=65521, a=17364, transform="korobov3")
        t, w = np.polynomial.legendre.leggauss(80)
        t, w = 0.5 * (t + 1), 0.5 * w
        grids = np.meshgrid(*([t] * d), indexing="ij")
        x = np.stack([g.ravel() for g in grids], axis=1)
        ww = np.ones(x.shape[0])
        for j in range(d):
            ww = ww * w[np.unravel_index(np.arange(x.shape[0]), (80,) * d)[j]]
        jac = 2 * x[:, 0]
        x[:, 0] = x[:, 0] ** 2
        ref = (ww[:, None] * jac[:, None] * oracle.integrand(sec, x)).sum(axis=0)
        mean, err = _integrate(sec)
        assert np.all(np.abs(mean - ref) < 5 * err + 1e-12)


def test_convergence_order_at_least_one():
    """RQMC error decays like n^(-alpha/2) with alpha >= 2 (Sec. 2.1.3)."""
    base = W.one_loop_sector(seed=0).sectors[0]
    ns = [(1009, 382), (4001, 1478), (16001, 6157), (64007, 24107)]
    errs = []
    for n, a in ns:
        sec = W.Sector(**{**base.__dict__, "n": n, "a": a})
        mean, err = _integrate(sec, m=16, seed=7)
        errs.append(err[0])
    slope = np.polyfit(np.log([n for n, _ in ns]), np.log(errs), 1)[0]
    assert slope < -1.0, (slope, errs)


@pytest.mark.parametrize("transform", ["none", "korobov3"])
def test_error_estimate_is_calibrated(transform):
    """The shift-based error (Sec. 2.1.3: standard error of the mean of m random-shift
    estimates) covers the exact value like a t-interval: over 200 independent shift sets
    with m = 16, |mean - exact| <= 2 err in about 94% of the cases (t with 15 degrees of
    freedom) and the standardised deviations have unit spread.  Integrand
    (1 + x1)^-1 (1 + x2)^-2 on a small lattice (n = 101), exact value log(2)/2."""
    sec = W.custom_sector(2, [(1, (0, 0)), (1, (1, 0))], [(1, (0, 0)), (1, (0, 1))],
                          u_pow=-1, f_pow2=-4, n=101, a=40, transform=transform)
    exact = math.log(2) / 2
    z = []
    for seed in range(200):
        sh = W.uniform_shifts(np.random.default_rng(1000 + seed), 16, 2)
        Q, _ = oracle.sector_sums(sec, sh)
        m, e = oracle.estimate(Q)
        z.append((m[0] - exact) / e[0])
    z = np.array(z)
    cover = np.mean(np.abs(z) <= 2.0)
    assert 0.86 <= cover <= 0.99, cover
    assert 0.8 <= np.std(z) <= 1.3 and abs(np.mean(z)) < 0.35


def test_zero_weight_samples_are_skipped_and_nonfinite_is_reported():
    # With korobov3, y = 0 gives W = 0: F = x1 vanishes there but the sample is skipped.
    sec = W.custom_sector(1, [], [(1, (1,))], f_pow2=-2, n=11, a=1, transform="korobov3")
    Q, _ = oracle.sector_sums(sec, np.zeros((2, 1)))
    assert np.all(np.isfinite(Q))
    # Without a transform the same point has weight 1 and 1/F is infinite.
    sec.transform = "none"
    with pytest.raises(oracle.OracleNonFinite, match="index 0"):
        oracle.sector_sums(sec, np.zeros((2, 1)))


# ---------------------------------------------------------------- summation

def test_neumaier_sum_is_compensated():
    assert oracle.neumaier([1.0, 1e100, 1.0, -1e100]) == 2.0
    v = np.array([1.0] + [1e-16] * 10000)
    assert oracle.neumaier(v) == 1.0 + 1e-12
    rng = np.random.default_rng(0)
    x = rng.normal(size=20000) * 10.0 ** rng.integers(-8, 8, size=20000)
    exact = math.fsum(x)
    assert abs(oracle.neumaier(x) - exact) <= 2 * abs(exact) * 2.0 ** -52


# ------------------------------------------------------------------ P_2

def _p2_dual_sum(n, z, H):
    """Truncated dual-lattice series sum_{0 != h in L^perp, |h_j| <= H} prod r(h_j)^-2."""
    z = [int(v) for v in z]
    inv3 = pow(z[2], -1, n)
    h = np.arange(-H, H + 1)
    r2 = np.maximum(1, np.abs(h)).astype(np.float64) ** -2
    tot = 0.0
    for i1, h1 in enumerate(h):
        res = (-(h1 * z[0] + h * z[1]) * inv3) % n          # h3 = res mod n, per h2
        for t in range(-(H // n) - 1, H // n + 2):
            h3 = res + t * n
            ok = np.abs(h3) <= H
            tot += r2[i1] * np.sum(r2[ok] * np.maximum(1, np.abs(h3[ok])) ** -2.0)
    return tot - 1.0     # remove h = 0


def test_p2_equals_dual_lattice_series():
    n = 101
    z = oracle.korobov_vector(n, 12, 3)
    p = oracle.p2(n, z)
    s1 = _p2_dual_sum(n, z, 400)
    s2 = _p2_dual_sum(n, z, 1600)
    # the tail of the series shrinks like 1/H: extrapolate and compare
    extrap = s2 + (s2 - s1) / 3.0
    assert abs(s2 - p) < 5e-3 * p
    assert abs(extrap - p) < 2e-5 * p


def test_p2_one_dimension_closed_form():
    # d = 1, z = 1: only h = multiples of n are dual, P2 = 2 zeta(2)/n^2 = pi^2/(3 n^2)
    for n in (7, 101, 65521):
        assert abs(oracle.p2(n, [1]) - math.pi ** 2 / (3 * n * n)) < 1e-9 * math.pi ** 2 / (3 * n * n) + 1e-15


def test_p2_symmetries_and_search_tie_rule():
    n = 1009
    for a in (5, 317, 600):
        p = oracle.p2(n, oracle.korobov_vector(n, a, 3))
        assert abs(oracle.p2(n, oracle.korobov_vector(n, n - a, 3)) - p) < 1e-13 * p
        ainv = pow(a, -1, n)
        assert abs(oracle.p2(n, oracle.korobov_vector(n, ainv, 3)) - p) < 1e-13 * p
    cands = list(range(2, 60))
    best, vals = oracle.korobov_search(n, 3, cands)
    assert best in cands
    assert vals[cands.index(best)] <= vals.min() * (1 + 1e-12)
    # brute-force argmin agrees up to the tie rule
    assert vals[cands.index(best)] == pytest.approx(vals.min(), rel=1e-12)


# --------------------------------------------------------------- statistics

def test_estimate_is_mean_and_standard_error():
    Q = np.array([[1.0, 10.0], [2.0, 10.0], [3.0, 10.0], [4.0, 10.0]])
    mean, err = oracle.estimate(Q)
    assert np.allclose(mean, [2.5, 10.0])
    assert np.allclose(err, [math.sqrt((5.0 / 3.0) / 4.0), 0.0])


def test_amplitude_variance_propagation_and_eps_rel():
    C = np.array([2.0 + 0j, -1.0 + 3.0j])
    ival = np.array([[1.0], [0.5]])
    ierr = np.array([[0.1], [0.2]])
    re, im, dre, dim = oracle.amplitude(C, ival, ierr)
    assert re[0] == pytest.approx(2.0 - 0.5)
    assert im[0] == pytest.approx(1.5)
    assert dre[0] == pytest.approx(math.sqrt(4 * 0.01 + 1 * 0.04))
    assert dim[0] == pytest.approx(math.sqrt(9 * 0.04))
    # Monte-Carlo check of the propagation rule with independent normal integrals
    rng = np.random.default_rng(0)
    samp = ival[:, 0][None, :] + ierr[:, 0][None, :] * rng.normal(size=(200000, 2))
    A = samp @ C
    assert np.std(A.real) == pytest.approx(dre[0], rel=0.01)
    assert np.std(A.imag) == pytest.approx(dim[0], rel=0.01)
    assert oracle.eps_rel(3.0, 4.0, 0.3, 0.4) == pytest.approx(0.1)
    # complex integrals (deformed contours): Re and Im of each integral independent
    iim = np.array([[-0.7], [0.4]])
    eim = np.array([[0.3], [0.05]])
    re, im, dre, dim = oracle.amplitude(C, ival, ierr, iim, eim)
    assert re[0] == pytest.approx(2.0 * 1.0 + (-1.0 * 0.5 - 3.0 * 0.4))
    assert im[0] == pytest.approx(2.0 * -0.7 + (-1.0 * 0.4 + 3.0 * 0.5))
    z = (ival[:, 0][None, :] + ierr[:, 0][None, :] * rng.normal(size=(200000, 2)) +
         1j * (iim[:, 0][None, :] + eim[:, 0][None, :] * rng.normal(size=(200000, 2))))
    A = z @ C
    assert np.std(A.real) == pytest.approx(dre[0], rel=0.01)
    assert np.std(A.imag) == pytest.approx(dim[0], rel=0.01)


def test_amplitude_series_is_the_product_of_series():
    # regulator-dependent coefficients (Sec. 2.4): the orders of A are the Cauchy product
    # of the coefficient's and the integrals' Laurent series (numpy's convolution), the
    # variance the sum over contributing terms with independent orders (Monte Carlo)
    rng = np.random.default_rng(4)
    NI, K, P = 3, 4, 3
    C = rng.normal(size=(NI, P)) + 1j * rng.normal(size=(NI, P))
    ival = rng.normal(size=(NI, K))
    ierr = rng.uniform(0.05, 0.3, size=(NI, K))
    re, im, dre, dim = oracle.amplitude_series(C, ival, ierr)
    want = sum(np.convolve(C[i], ival[i])[:K] for i in range(NI))
    assert np.allclose(re, want.real, rtol=1e-13, atol=1e-13)
    assert np.allclose(im, want.imag, rtol=1e-13, atol=1e-13)
    samp = ival[None] + ierr[None] * rng.normal(size=(100000, NI, K))
    # the convolution with c_i as a lower-triangular Toeplitz matrix
    Tm = np.zeros((NI, K, K), dtype=np.complex128)
    for i in range(NI):
        for j in range(K):
            for p in range(min(P, j + 1)):
                Tm[i, j, j - p] = C[i, p]
    A = np.einsum("sik,ijk->sj", samp, Tm)
    assert np.allclose(np.std(A.real, axis=0), dre, rtol=0.02)
    assert np.allclose(np.std(A.imag, axis=0), dim, rtol=0.02)
    # one constant term reduces to the per-order rule
    r1 = oracle.amplitude_series(C[:, :1], ival, ierr)
    r0 = oracle.amplitude(C[:, 0], ival, ierr)
    for a, b in zip(r1, r0):
        assert np.allclose(a, b, rtol=1e-14)


# --------------------------------------------------------------- allocation

def test_allocation_satisfies_constraint_and_stationarity():
    rng = np.random.default_rng(2)
    for alpha in (2.0, 3.0):
        c2 = rng.uniform(0.1, 5, size=7)
        w = rng.uniform(1e-3, 1, size=7)
        tau = rng.uniform(1, 10, size=7)
        V = 1e-8
        n, lam = oracle.allocate(c2, w, tau, V, alpha)
        assert np.sum(c2 * w / n ** alpha) == pytest.approx(V, rel=1e-12)
        # dT/dn_i + lambda d var/dn_i = tau_i - lambda alpha c2_i w_i n_i^(-alpha-1) = 0
        assert np.allclose(tau, lam * alpha * c2 * w * n ** (-alpha - 1), rtol=1e-12)


def test_allocation_is_the_constrained_minimum():
    c2 = np.array([1.0, 4.0, 0.25])
    w = np.array([0.5, 0.1, 2.0])
    tau = np.array([1.0, 3.0, 0.5])
    V = 1e-6
    n, _ = oracle.allocate(c2, w, tau, V)
    # brute force: minimise sum tau n subject to the variance constraint (log variables)
    cons = {"type": "eq", "fun": lambda u: np.log(np.sum(c2 * w * np.exp(-2 * u)) / V)}
    res = optimize.minimize(lambda u: np.sum(tau * np.exp(u)) / np.sum(tau * n), np.log(n) + 0.3,
                            constraints=[cons], method="SLSQP", options={"ftol": 1e-14,
                                                                         "maxiter": 500})
    assert res.success
    assert np.allclose(np.exp(res.x), n, rtol=1e-4)
    # any feasible perturbation costs more
    for _ in range(20):
        u = np.log(n) + np.random.default_rng(_).normal(scale=0.1, size=3)
        scale = (np.sum(c2 * w * np.exp(-2 * u)) / V) ** 0.5
        u = u + np.log(scale)
        assert np.sum(tau * np.exp(u)) >= np.sum(tau * n) * (1 - 1e-12)


def test_splitmix64_reference_values():
    # First outputs of the published generator with state 0 (Steele-Lea-Flood 2014).
    assert oracle.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert oracle.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert oracle.splitmix64(0, 2) == 0x06C45D188009454F


def test_median_rule_picks_the_middle_estimate():
    # Sec. 2.2, Eq. median: the median of r unshifted lattice estimates, each the plain
    # rank-1 rule with its candidate vector; r = 1 is the candidate itself
    sec = W.custom_sector(2, [(1.0, (0, 0))], [(1.0, (0, 0)), (1.0, (1, 1))], f_pow2=-2,
                          logc=[[1.0]], transform="korobov3", n=1009)
    exact = math.pi ** 2 / 12
    rng = np.random.default_rng(0)
    cands = W.median_candidates(rng, 1009, 2, 15)
    assert np.all(np.gcd(cands.astype(np.int64), 1009) == 1) and cands.min() >= 1
    c, Q = oracle.median_rule(sec, 1009, cands)
    vals = Q[:, 0]
    assert vals[c] == np.sort(vals)[7]                     # the middle of 15
    assert np.all(np.abs(vals - exact) < 1e-2)             # every candidate is a lattice rule
    # each candidate's estimate is the unshifted lattice rule with that vector
    z = cands[3]
    direct = oracle.sector_sums(sec, np.zeros((1, 2)), n=1009, z=z)[0][0, 0]
    assert Q[3, 0] == direct
    c1, Q1 = oracle.median_rule(sec, 1009, cands[:1])
    assert c1 == 0 and Q1[0, 0] == Q[0, 0]
    # even r: the lower middle
    c4, Q4 = oracle.median_rule(sec, 1009, cands[:4])
    assert Q4[c4, 0] == np.sort(Q4[:, 0])[1]
