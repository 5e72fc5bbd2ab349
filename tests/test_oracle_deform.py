"""Pins of the oracle's contour-deformed integrand (CPU only).

The deformed estimator is pinned by what the mathematics fixes independently of it:
  * the one-loop bubble above threshold, whose F - i0 integrals are known in closed
    form (real and imaginary parts, so the branch and the sign of the deformation are
    checked);
  * Cauchy's theorem: on Euclidean integrands (F > 0 on the cube) the deformed integral
    equals the undeformed closed form, which fails for a wrong Jacobian, a wrong
    gradient, or a monomial or U left undeformed;
  * the Jacobian determinant against central finite differences of z(x), and z, F(z)
    against the polynomial written out at complex points;
  * the sign check (Im F(z) <= 0) and the presample halving of lambda.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

ZETA3 = 1.2020569031595942


def _lattice(n):
    cands = np.arange(2, min(n - 1, 400), dtype=np.uint64)
    return oracle.korobov_search(n, 2, cands)[0]


def _estimate(sec, m=8, seed=0, lam=None):
    rng = np.random.default_rng(seed)
    shifts = W.uniform_shifts(rng, m, sec.d)
    Q, _, viol, _ = oracle.sector_sums_deformed(sec, shifts, lam=lam, threads=8)
    assert viol == 0
    return oracle.estimate(Q.real) + oracle.estimate(Q.imag)


def test_jacobian_and_map_against_definitions():
    rng = np.random.default_rng(5)
    d = 3
    terms = [(0.7, (0, 0, 0))] + [(float(rng.uniform(-2, 2)), tuple(int(v) for v in e))
                                  for e in rng.integers(0, 3, size=(8, d))]
    sec = W.custom_sector(d, [(1.0, (0, 0, 0))], terms)
    lam = 0.4
    fe = np.array([t[1] for t in terms], dtype=float)
    fc = np.array([t[0] for t in terms])

    def F_def(x):        # F written out at a real or complex point
        return np.sum(fc * np.prod(np.asarray(x)[None, :] ** fe, axis=1))

    for x in rng.uniform(0.05, 0.95, size=(6, d)):
        z, J, Fz = oracle.deform_point(sec, x[None, :], lam)
        z, J, Fz = z[0], J[0], Fz[0]
        h = 1e-6
        grad = np.array([(F_def(x + h * e) - F_def(x - h * e)) / (2 * h) for e in np.eye(d)])
        assert np.allclose(z.real, x, rtol=0, atol=0)
        assert np.allclose(z.imag, -lam * x * (1 - x) * grad, rtol=1e-7, atol=1e-9)
        assert abs(Fz - F_def(z)) <= 1e-12 * (1 + abs(Fz))
        # dz/dx by central differences of the oracle's own map, then its determinant
        Jm = np.empty((d, d), dtype=complex)
        for k in range(d):
            e = np.zeros(d)
            e[k] = h
            zp = oracle.deform_point(sec, (x + e)[None, :], lam)[0][0]
            zm = oracle.deform_point(sec, (x - e)[None, :], lam)[0][0]
            Jm[:, k] = (zp - zm) / (2 * h)
        assert abs(J - np.linalg.det(Jm)) <= 1e-6 * abs(J)


@pytest.mark.parametrize("kind", ["inverse", "log"])
def test_bubble_above_threshold_closed_form(kind):
    # F = m^2 - s x (1 - x), s > 4 m^2: both roots inside (0, 1).  With beta^2 = 1 - 4 m^2/s,
    #   int_0^1 dx / (F - i0)  = 2/(s beta) [log((1 - beta)/(1 + beta)) + i pi]
    #   int_0^1 log(F - i0) dx = log m^2 - 2 + beta log((1 + beta)/(1 - beta)) - i pi beta
    s, m2 = 10.0, 1.0
    beta = math.sqrt(1 - 4 * m2 / s)
    f_terms = [(m2, (0,)), (-s, (1,)), (s, (2,))]
    if kind == "inverse":
        sec = W.custom_sector(1, [(1.0, (0,))], f_terms, f_pow2=-2, logc=[[1.0]],
                              transform="korobov3", n=100003)
        exact = 2 / (s * beta) * (math.log((1 - beta) / (1 + beta)) + 1j * math.pi)
    else:
        sec = W.custom_sector(1, [(1.0, (0,))], f_terms, logc=[[0.0, 1.0]],
                              transform="korobov3", n=100003)
        exact = (math.log(m2) - 2 + beta * math.log((1 + beta) / (1 - beta))
                 - 1j * math.pi * beta)
    rng = np.random.default_rng(1)
    shifts = W.uniform_shifts(rng, 8, 1)
    lam, _ = oracle.choose_lambda(sec, shifts, 0.5, 1009, 1)
    Q, _, viol, _ = oracle.sector_sums_deformed(sec, shifts, a=1, lam=lam, threads=8)
    assert viol == 0
    mr, er = oracle.estimate(Q.real)
    mi, ei = oracle.estimate(Q.imag)
    assert abs(mr[0] - exact.real) <= 6 * er[0] + 1e-9
    assert abs(mi[0] - exact.imag) <= 6 * ei[0] + 1e-9
    assert er[0] < 1e-6 and ei[0] < 1e-6


def test_cauchy_invariance_two_dimensional():
    # F = 1 + x y > 0: the deformed integrals equal int int (1+xy)^-1 {1, log(1+xy)}
    sec = W.custom_sector(2, [(1.0, (0, 0))], [(1.0, (0, 0)), (1.0, (1, 1))], f_pow2=-2,
                          logc=[[1.0, 0.0], [0.0, 1.0]], transform="korobov3", n=32749,
                          deform_lambda=0.5)
    sec.a = _lattice(sec.n)
    rng = np.random.default_rng(2)
    shifts = W.uniform_shifts(rng, 8, 2)
    Q, _, viol, _ = oracle.sector_sums_deformed(sec, shifts, threads=8)
    assert viol == 0
    mr, er = oracle.estimate(Q.real)
    mi, ei = oracle.estimate(Q.imag)
    exact = np.array([math.pi ** 2 / 12, ZETA3 / 8])
    assert np.all(np.abs(mr - exact) <= 6 * er + 1e-10)
    assert np.all(np.abs(mi) <= 6 * ei + 1e-10)
    # and the deformation is really there: the per-point imaginary parts are not small
    x = np.array([[0.3, 0.6]])
    assert abs(oracle.deform_point(sec, x)[1][0].imag) > 0.05


@pytest.mark.parametrize("case", ["half_power", "u_power"])
def test_cauchy_invariance_monomial_and_u(case):
    # int_0^1 sqrt(x)/(1+x) = 2 - pi/2 (x^(1/2) must be deformed too);
    # int_0^1 (1+x)^-1 (1+x)^-1 = 1/2 with U = 1 + x taken at z
    if case == "half_power":
        sec = W.custom_sector(1, [(1.0, (0,))], [(1.0, (0,)), (1.0, (1,))], x_pow2=[1],
                              f_pow2=-2, transform="korobov3", n=65537, deform_lambda=0.5)
        exact = 2 - math.pi / 2
    else:
        sec = W.custom_sector(1, [(1.0, (0,)), (1.0, (1,))], [(1.0, (0,)), (1.0, (1,))],
                              u_pow=-1, f_pow2=-2, transform="korobov3", n=65537,
                              deform_lambda=0.5)
        exact = 0.5
    rng = np.random.default_rng(3)
    shifts = W.uniform_shifts(rng, 8, 1)
    Q, _, viol, _ = oracle.sector_sums_deformed(sec, shifts, a=1, threads=8)
    assert viol == 0
    mr, er = oracle.estimate(Q.real)
    mi, ei = oracle.estimate(Q.imag)
    assert abs(mr[0] - exact) <= 6 * er[0] + 1e-11
    assert abs(mi[0]) <= 6 * ei[0] + 1e-11
    # undeformed monomial would give a visibly different value
    z, J, _ = oracle.deform_point(sec, np.array([[0.5]]))
    assert abs(z[0, 0] - 0.5) > 0.1


def test_sign_check_and_presample_lambda():
    # cubic physical F: a large lambda turns Im F(z) positive somewhere, halving fixes it
    f = [(1.0, (0, 0)), (-6.0, (1, 0)), (6.0, (2, 0)), (-3.0, (1, 1)), (4.0, (3, 0)),
         (2.0, (0, 3))]
    sec = W.custom_sector(2, [(1.0, (0, 0))], f, f_pow2=-2, transform="korobov3", n=1009,
                          a=76)
    rng = np.random.default_rng(0)
    sh = W.uniform_shifts(rng, 4, 2)
    assert oracle.sign_violations(sec, sh, 4.0, 1009, 76) > 0
    lam, halvings = oracle.choose_lambda(sec, sh, 4.0, 1009, 76)
    assert halvings >= 1 and lam == 4.0 / 2 ** halvings
    assert oracle.sign_violations(sec, sh, lam, 1009, 76) == 0
    assert oracle.sign_violations(sec, sh, 2 * lam, 1009, 76) > 0
    # the summation reports the same violations it finds
    sec.deform_lambda = 4.0
    Q, S, viol, first = oracle.sector_sums_deformed(sec, sh)
    assert viol == oracle.sign_violations(sec, sh, 4.0, 1009, 76) and first is not None
    with pytest.raises(oracle.OracleSignCheck):
        oracle.sector_sums(sec, sh)
    # Euclidean F never violates at the default lambda
    euc = W.custom_sector(2, [(1.0, (0, 0))], [(1.0, (0, 0)), (1.0, (1, 1)), (0.5, (2, 1))],
                          f_pow2=-2, transform="korobov3", n=1009, a=76)
    assert oracle.sign_violations(euc, sh, 0.5, 1009, 76) == 0


def test_branch_of_f_minus_i0_on_the_real_contour():
    # lambda = 0 on F = x - 1/2: int_0^1 log(F - i0) = int log|x - 1/2| - i pi * (1/2)
    #                                                 = -1 - log 2 - i pi / 2
    sec = W.custom_sector(1, [(1.0, (0,))], [(-0.5, (0,)), (1.0, (1,))], logc=[[0.0, 1.0]],
                          transform="none", n=100003)
    rng = np.random.default_rng(4)
    shifts = W.uniform_shifts(rng, 8, 1)
    Q, _, viol, _ = oracle.sector_sums_deformed(sec, shifts, a=1, lam=0.0)
    assert viol == 0
    mr, _ = oracle.estimate(Q.real)
    mi, _ = oracle.estimate(Q.imag)
    assert abs(mr[0] - (-1 - math.log(2))) < 1e-3           # log singularity: slow, but close
    assert abs(mi[0] + math.pi / 2) < 1e-4                    # -i pi on the half where F < 0
