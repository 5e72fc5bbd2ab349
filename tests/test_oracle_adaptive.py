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


def fine_ladder(seed=0):
    """Lattice sizes 5% apart (so the ceiling of a requested size is close to it)."""
    sizes, cands = W.lattice_ladder(n_min=1009, n_max=3_000_000, ratio=1.05, n_cand=1, seed=seed)
    return sizes, cands[:, :, 0]


def series_coefficients():
    """One sum over the three closed-form integrals with two Laurent terms per coefficient
    (eps^0 and eps^1, Sec. 2.4), so that order k of the sum also draws on order k - 1 of
    the integrals."""
    return np.array([[[2.0, 0.7], [-0.5 + 0.25j, 0.3j], [1.5j, -0.4]]])


def check_allocation_round_properties(ora):
    """Every allocation decision of the adaptive loop against what the optimum of Sec.
    2.1.3 must satisfy, using only what the round measured (per-sector standard errors
    err_s,k at the integrated sizes n_s) and the costs tau_s:
      * the variance model (Eq. varscaling): sector s contributes
        w_s = sum_p |c_p|^2 err_s,k-p^2 n_s^alpha / n^alpha at size n, so the predicted
        variance of the target at the closed-form sizes, sum_s w_s / n_opt_s^alpha, equals
        the bound V (before the never-shrink maximum and the ladder ceiling);
      * stationarity of the Lagrangian sum_s tau_s n_s + lambda (sum_s w_s/n_s^alpha - V):
        tau_s n_opt_s^(alpha + 1) / w_s is the same for every contributing sector;
      * a sector contributes exactly when its w_s > 0.
    None of these restates how the loop computes its sizes: a wrong power of the error,
    an order offset, the integral's variance in place of the sector's or a missing
    |c|^2 moves n_opt off both surfaces."""
    prob, _ = closed_form_problem()
    C = series_coefficients()
    sizes, a_tab = fine_ladder()
    tau = np.array([1.0, 1.5, 1.0, 3.0, 2.0, 0.5])
    alpha = 2.0
    trace = []
    val, err, nfin, rounds, conv = ora.adaptive_amplitude(prob, C, sizes, a_tab, tau,
                                                          epsrel=3e-10, n_presample=1009,
                                                          alpha=alpha, trace=trace)
    assert len(trace) == rounds
    P = C.shape[2]
    checked = set()
    for rec in trace:
        for tg in rec["targets"]:
            t, k, V, n_opt = tg["t"], tg["k"], tg["V"], tg["n_opt"]
            w = np.zeros(len(prob.sectors))
            for s, sec in enumerate(prob.sectors):
                c = C[t, sec.integral]
                w[s] = sum(abs(c[p]) ** 2 * rec["err"][s, k - p] ** 2
                           for p in range(min(P, k + 1))) * rec["n"][s] ** alpha
            use = w > 0
            assert np.array_equal(use, n_opt > 0), (use, n_opt)
            pred = float(np.sum(w[use] / n_opt[use] ** alpha))
            assert abs(pred - V) <= 1e-9 * V, (pred, V)
            r = rec["tau"][use] * n_opt[use] ** (alpha + 1) / w[use]
            assert np.allclose(r, r[0], rtol=1e-9, atol=0), r
            checked.add(k)
    assert checked == {0, 1}, checked   # both orders, the second with the eps^1 term
    return trace


def test_allocation_round_properties():
    check_allocation_round_properties(oracle)


def check_allocation_converges_to_truth_with_series(ora):
    """The series-coefficient sum reaches its target and the truth (the Cauchy product of
    the coefficient series with the exact integrals)."""
    prob, exact = closed_form_problem()
    C = series_coefficients()
    sizes, a_tab = fine_ladder()
    tau = np.array([1.0, 1.5, 1.0, 3.0, 2.0, 0.5])
    val, err, nfin, rounds, conv = ora.adaptive_amplitude(prob, C, sizes, a_tab, tau,
                                                          epsrel=3e-10, n_presample=1009)
    truth = np.zeros(2, dtype=complex)
    for i in range(3):
        truth[0] += C[0, i, 0] * exact[i, 0]
        truth[1] += C[0, i, 0] * exact[i, 1] + C[0, i, 1] * exact[i, 0]
    assert conv and rounds >= 2
    assert np.all(np.abs(err[0]) / np.abs(val[0]) <= 3e-10)
    assert np.all(np.abs(val[0] - truth) <= 6 * np.abs(err[0]) + 1e-14), (val, truth, err)


def test_allocation_converges_to_truth_with_series():
    check_allocation_converges_to_truth_with_series(oracle)


def test_measured_costs_per_round_are_used_in_order():
    """tau given per round ([R, S]): the allocation after round r uses row r - 1 (the last
    row afterwards), as the trace records."""
    prob, _ = closed_form_problem()
    sizes, a_tab = fine_ladder()
    rows = np.array([[1.0, 1.0, 1.0, 1.0, 2.0, 2.0], [3.0, 1.0, 2.0, 1.0, 1.0, 0.5]])
    trace = []
    oracle.adaptive_amplitude(prob, np.array([[1.0, 1.0, 1.0]]), sizes, a_tab, rows,
                              epsrel=1e-10, n_presample=1009, trace=trace)
    assert len(trace) >= 2
    for r, rec in enumerate(trace):
        assert np.array_equal(rec["tau"], rows[min(r, 1)])
