"""Pins of the oracle's adaptive weighted-sum evaluation (Sec. 2.1.3) on integrals with
closed forms: the final estimate must lie within a few reported standard errors of the
exact amplitude and meet the requested relative error."""
import math

import numpy as np

import oracle
import workloads as W

ZETA3 = 1.2020569031595942


def closed_form_problem(m=8):
    """Three integrals with K = 2 orders each, every integral split over two sectors:
    I1 = int (1+x)^-3 {1, log(1+x)}               = {3/8, 3/16 - log(2)/8}
    I2 = int_0^1 {1, -log F}, F = t/2 - t^2/4 (bubble) = {1, 2}
    I3 = int int (1+x y)^-1 {1, log(1+x y)}        = {pi^2/12, zeta(3)/8}"""
    secs = []
    for c in (0.3, 0.7):
        secs.append(W.custom_sector(1, [(c, (0,))], [(1.0, (0,)), (1.0, (1,))], u_pow=1, f_pow2=-6,
                                    logc=[[1, 0], [0, 1]], transform="korobov3", integral=0))
    for c in (0.25, 0.75):
        secs.append(W.custom_sector(1, [(c, (0,))], [(0.5, (1,)), (-0.25, (2,))], u_pow=1,
                                    logc=[[1, 0], [0, -1]], transform="korobov3", integral=1))
    for c in (0.6, 0.4):
        secs.append(W.custom_sector(2, [(c, (0, 0))], [(1.0, (0, 0)), (1.0, (1, 1))], u_pow=1,
                                    f_pow2=-2, logc=[[1, 0], [0, 1]], transform="korobov3",
                                    integral=2))
    rng = np.random.default_rng(4)
    shifts = [W.uniform_shifts(rng, m, s.d) for s in secs]
    prob = W.Problem(sectors=secs, order_lo=0, m=m, shifts=shifts, n_integrals=3)
    exact = np.array([[3 / 8, 3 / 16 - math.log(2) / 8], [1.0, 2.0],
                      [math.pi ** 2 / 12, ZETA3 / 8]])
    return prob, exact


def ladder(seed=0):
    sizes, cands = W.lattice_ladder(n_min=1009, n_max=300000, ratio=1.6, n_cand=1, seed=seed)
    return sizes, cands[:, :, 0]


def test_adaptive_amplitude_reaches_target_and_truth():
    prob, exact = closed_form_problem()
    coef = np.array([[2.0, -0.5 + 0.25j, 1.5j]])
    sizes, a_tab = ladder()
    tau = np.array([1.0, 1.0, 1.0, 1.0, 2.0, 2.0])
    val, err, nfin, rounds, conv = oracle.adaptive_amplitude(prob, coef, sizes, a_tab, tau,
                                                             epsrel=1e-9, n_presample=1009)
    truth = coef[0] @ exact
    assert conv and rounds >= 2
    rel = np.abs(err[0]) / np.abs(val[0])
    assert np.all(rel <= 1e-9)
    dev = np.abs(val[0] - truth)
    assert np.all(dev <= 6 * np.abs(err[0]) + 1e-14), (dev, err)
    # lattices only grow from the presample size and stay in the table
    assert all(int(n) in set(int(s) for s in sizes) for n in nfin)
    assert nfin.min() >= 1009


def test_adaptive_amplitude_allocates_towards_the_expensive_noisy_units():
    prob, _ = closed_form_problem()
    coef = np.array([[1.0, 1.0, 1.0]])
    sizes, a_tab = ladder()
    cheap = np.ones(6)
    costly = np.array([1.0, 1.0, 1.0, 1.0, 50.0, 50.0])
    _, _, n1, _, _ = oracle.adaptive_amplitude(prob, coef, sizes, a_tab, cheap, epsrel=1e-10,
                                               n_presample=1009)
    _, _, n2, _, _ = oracle.adaptive_amplitude(prob, coef, sizes, a_tab, costly, epsrel=1e-10,
                                               n_presample=1009)
    # raising a unit's cost never raises its share of the lattice points
    assert n2[4] <= n1[4] and n2[5] <= n1[5]


def test_single_round_when_presample_already_meets_target():
    prob, _ = closed_form_problem()
    sizes, a_tab = ladder()
    val, err, nfin, rounds, conv = oracle.adaptive_amplitude(
        prob, np.array([[1.0, 0.0, 0.0]]), sizes, a_tab, np.ones(6), epsrel=1e-2,
        n_presample=1009)
    assert conv and rounds == 1 and np.all(nfin == sizes[0])
