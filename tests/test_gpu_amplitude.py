"""GPU parity of amp_evaluate (adaptive weighted sums, Sec. 2.1.3) with the oracle's
adaptive loop: same lattice table, costs and shifts give the same rounds and final
lattice sizes, and sums within 1e-12 of the oracle's on their scale."""
import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle_adaptive import closed_form_problem, ladder

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qmc():
    import __graft_entry__ as g
    g._ensure_built()
    import torch
    import paper_2305_19768_amd as q
    torch.cuda.set_device(0)
    return q


def _compare(qmc, prob, coef, sizes, a_tab, tau, epsrel, n_presample, persistent=False, **kw):
    plan = qmc.Plan(prob, n_max=int(sizes[-1]))
    if persistent:   # the batched form's persistent kernel specialised to the plan
        plan.specialize(persistent=True)
    val, err, nfin, st = plan.amp_evaluate(coef, epsrel=epsrel, lattice_n=sizes, lattice_a=a_tab,
                                           tau=tau, n_presample=n_presample, **kw)
    ov, oe, on, orounds, oconv = oracle.adaptive_amplitude(prob, coef, sizes, a_tab, tau,
                                                           epsrel=epsrel, n_presample=n_presample)
    print("rounds", st["rounds"], orounds, "n", nfin, on, flush=True)
    assert st["rounds"] == orounds
    assert bool(st["converged"]) == oconv
    assert np.array_equal(nfin, on)
    scale = np.abs(ov) + np.abs(oe)
    assert np.all(np.abs(val - ov) <= 1e-12 * scale)
    assert np.allclose(err.real, oe.real, rtol=1e-8, atol=1e-12 * np.max(scale))
    assert np.allclose(err.imag, oe.imag, rtol=1e-8, atol=1e-12 * np.max(scale))
    return val, err, nfin, st


@pytest.mark.parametrize("mode", [0, 1])
def test_closed_form_amplitude_parity(qmc, mode):
    prob, exact = closed_form_problem()
    coef = np.array([[2.0, -0.5 + 0.25j, 1.5j]])
    sizes, a_tab = ladder()
    tau = np.array([1.0, 1.0, 1.0, 1.0, 2.0, 2.0])
    val, err, nfin, st = _compare(qmc, prob, coef, sizes, a_tab, tau, 1e-9, 1009, mode=mode)
    assert st["converged"] and st["evaluations"] > 0
    assert np.all(np.abs(val[0] - coef[0] @ exact) <= 6 * np.abs(err[0]) + 1e-14)


@pytest.mark.parametrize("mode", [0, 1])
def test_synthetic_amplitude_parity(qmc, mode):
    prob = W.amplitude(seed=1, n_integrals=6, n_sectors=24, d_lo=3, d_hi=6, m=8, n0=1009)
    sizes, a_tab = ladder(seed=2)
    tau = np.array([float(s.d) for s in prob.sectors])
    coef = np.array([prob.amp_coef, prob.amp_coef * (0.5 - 1j)])   # two sums, in order
    _compare(qmc, prob, coef, sizes, a_tab, tau, 2e-6, 1009, mode=mode)



@pytest.mark.parametrize("fp32", [False, True])
def test_device_mode_repeated_calls_are_identical(qmc, fp32):
    # the batched form builds its tables in a host image kept by the plan: a second call
    # on the same plan, after a call on another plan with fewer sectors and sums, gives
    # the same rounds, lattices, sums and errors bit for bit
    prob = W.amplitude(seed=1, n_integrals=6, n_sectors=24, d_lo=3, d_hi=6, m=8, n0=1009)
    small = W.amplitude(seed=4, n_integrals=3, n_sectors=9, d_lo=3, d_hi=5, m=8, n0=1009)
    sizes, a_tab = ladder(seed=2)
    prec = qmc.QMC_PREC_FP32 if fp32 else qmc.QMC_PREC_FP64
    coef = np.array([prob.amp_coef, prob.amp_coef * (0.5 - 1j)])
    tau = np.array([float(s.d) for s in prob.sectors])
    plan = qmc.Plan(prob, precision=prec, n_max=int(sizes[-1]))
    other = qmc.Plan(small, precision=prec, n_max=int(sizes[-1]))
    kw = dict(epsrel=2e-6, lattice_n=sizes, lattice_a=a_tab, n_presample=1009, mode=1)
    first = plan.amp_evaluate(coef, tau=tau, **kw)
    o = other.amp_evaluate(np.array([small.amp_coef]),
                           tau=np.array([float(s.d) for s in small.sectors]), **kw)
    assert np.all(np.isfinite(o[0]))
    second = plan.amp_evaluate(coef, tau=tau, **kw)
    print("rounds", first[3]["rounds"], second[3]["rounds"], flush=True)
    assert first[3]["rounds"] == second[3]["rounds"]
    assert first[3]["evaluations"] == second[3]["evaluations"]
    for a, b in zip(first[:3], second[:3]):
        assert np.array_equal(a, b)

def _series_coefficients(qmc, exprs, symbols, K):
    """Laurent terms of the coefficient expressions from the library's exact expansion,
    checked bit for bit against the oracle's exact rational functions."""
    from oracle import coef as OC
    leads = [qmc.coef_series(e, symbols=symbols, n_terms=0)[0] for e in exprs]
    lo = min(l for l in leads if l is not None)
    C = np.zeros((len(exprs), K), dtype=np.complex128)
    for i, e in enumerate(exprs):
        C[i] = qmc.coef_series(e, symbols=symbols, order_lo=lo, n_terms=K)[1]
        want = [OC.to_complex(t) for t in OC.series(e, symbols=symbols, order_lo=lo, n_terms=K)[1]]
        assert list(C[i]) == want
    return C, lo


@pytest.mark.parametrize("mode", [0, 1])
def test_regulator_dependent_coefficients_parity(qmc, mode):
    # coefficients with poles and zeros in eps (d = 4 - 2 eps): the sums are products of
    # series; same rounds, final lattices and values as the oracle's loop
    prob = W.amplitude(seed=1, n_integrals=6, n_sectors=24, d_lo=3, d_hi=6, m=8, n0=1009)
    exprs, symbols = W.coefficient_expressions(seed=5, n_integrals=6)
    C, lo = _series_coefficients(qmc, exprs, symbols, prob.K)
    assert lo == -1
    sizes, a_tab = ladder(seed=2)
    tau = np.array([float(s.d) for s in prob.sectors])
    coef = np.stack([C, 0.5j * C])                  # two sums, [T, NI, P]
    _compare(qmc, prob, coef, sizes, a_tab, tau, 2e-6, 1009, mode=mode, coef_order_lo=lo)


def test_named_sums_from_expressions(qmc):
    # named, sparse and dense rows of expressions give the same sums as the numeric route
    prob = W.amplitude(seed=1, n_integrals=6, n_sectors=24, d_lo=3, d_hi=6, m=8, n0=1009)
    exprs, symbols = W.coefficient_expressions(seed=5, n_integrals=6)
    sizes, a_tab = ladder(seed=2)
    tau = np.array([float(s.d) for s in prob.sectors])
    plan = qmc.Plan(prob, n_max=int(sizes[-1]))
    sums = {"dense": exprs, "sparse": {0: exprs[0], 3: f"I*({exprs[3]})"}}
    out, nfin, st = plan.amp_evaluate_expressions(sums, symbols, epsrel=2e-6, lattice_n=sizes,
                                                  lattice_a=a_tab, tau=tau, n_presample=1009)
    C, lo = _series_coefficients(qmc, exprs, symbols, prob.K)
    Cs = np.zeros_like(C)
    Cs[0], Cs[3] = C[0], 1j * C[3]
    ov, oe, on, orounds, _ = oracle.adaptive_amplitude(prob, np.stack([C, Cs]), sizes, a_tab,
                                                       tau, epsrel=2e-6, n_presample=1009)
    assert out["dense"]["orders"] == [prob.order_lo + lo + j for j in range(prob.K)]
    assert st["rounds"] == orounds and np.array_equal(nfin, on)
    for t, name in enumerate(("dense", "sparse")):
        scale = np.abs(ov[t]) + np.abs(oe[t])
        assert np.all(np.abs(out[name]["value"] - ov[t]) <= 1e-12 * scale)


def test_device_mode_fp32_meets_target(qmc):
    # batched form with the FP32 integrand: same target met, values within FP32 bar of oracle
    prob = W.amplitude(seed=1, n_integrals=6, n_sectors=24, d_lo=3, d_hi=6, m=8, n0=1009)
    sizes, a_tab = ladder(seed=2)
    tau = np.array([float(s.d) for s in prob.sectors])
    plan = qmc.Plan(prob, n_max=int(sizes[-1]), precision=qmc.QMC_PREC_FP32)
    val, err, nfin, st = plan.amp_evaluate(prob.amp_coef, epsrel=5e-4, lattice_n=sizes,
                                           lattice_a=a_tab, tau=tau, n_presample=1009, mode=1)
    assert st["converged"] == 1
    rel = np.abs(err[0]) / np.abs(val[0])
    assert np.all(rel <= 5e-4)
    ov, oe, on, _, _ = oracle.adaptive_amplitude(prob, prob.amp_coef, sizes, a_tab, tau,
                                                 epsrel=5e-4, n_presample=1009)
    # both estimates of the same amplitude agree within their combined errors
    assert np.all(np.abs(val[0] - ov[0]) <= 5 * (np.abs(err[0]) + np.abs(oe[0])))


@pytest.mark.parametrize("fp32", [False, True])
def test_device_mode_with_flow_sectors_matches_host_mode(qmc, fp32):
    # flows attached to three sectors: the batched form integrates them in the flow
    # persistent kernel beside the plain sectors; same rounds and lattices as the host
    # loop, sums equal to rounding order
    from oracle import flow as OF
    prob = W.amplitude(seed=1, n_integrals=6, n_sectors=24, d_lo=3, d_hi=6, m=8, n0=1009)
    sizes, a_tab = ladder(seed=2)
    tau = np.array([float(s.d) for s in prob.sectors])
    prec = qmc.QMC_PREC_FP32 if fp32 else qmc.QMC_PREC_FP64
    out = {}
    for mode in (qmc.QMC_AMP_HOST, qmc.QMC_AMP_DEVICE):
        plan = qmc.Plan(prob, n_max=int(sizes[-1]), precision=prec)
        flows = []
        for s in (1, 5, 9):
            d = prob.sectors[s].d
            p = OF.init_params(d, seed=30 + s, zero_last=False, scale=0.7)
            fl = qmc.flow.Flow(d, params=OF.flatten(p))
            plan.attach_flow(s, fl)
            flows.append(fl)
        out[mode] = plan.amp_evaluate(prob.amp_coef, epsrel=2e-6, lattice_n=sizes,
                                      lattice_a=a_tab, tau=tau, n_presample=1009, mode=mode)
        del plan
    vh, eh, nh, sh = out[qmc.QMC_AMP_HOST]
    vd, ed, nd, sd = out[qmc.QMC_AMP_DEVICE]
    print("rounds", sh["rounds"], sd["rounds"], "n", nh, nd, flush=True)
    assert sd["rounds"] == sh["rounds"] and np.array_equal(nd, nh)
    assert sd["evaluations"] == sh["evaluations"]
    scale = np.abs(vh) + np.abs(eh)
    assert np.all(np.abs(vd - vh) <= 1e-12 * scale)
    assert np.allclose(ed.real, eh.real, rtol=1e-8, atol=1e-12 * np.max(scale))


def test_device_mode_with_more_sectors_than_round_threads(qmc):
    # 600 sectors: each thread of the round kernel takes a run of two or three sectors
    # when it lays out the next round's workgroups; rounds, final lattices and sums as
    # in the oracle's adaptive loop
    prob = W.amplitude(seed=4, n_integrals=12, n_sectors=600, d_lo=2, d_hi=4, m=4, n0=1009)
    sizes, a_tab = ladder(seed=3)
    tau = np.array([float(s.d) for s in prob.sectors])
    val, err, nfin, st = _compare(qmc, prob, np.array([prob.amp_coef]), sizes, a_tab, tau, 1e-5,
                                  1009, mode=1)
    assert st["rounds"] >= 3 and np.count_nonzero(nfin > 1009) > 100


@pytest.mark.parametrize("mixed", [False, True])
def test_device_mode_fp32_against_fp64(qmc, mixed):
    # The FP32 batched form against the FP64 one on the same ladder: same rounds and final
    # lattices, sums within the FP32 bar on their scale.  mixed: one sector's F gets a
    # negative coefficient (F stays positive on the cube), so it has no FP32 form and the
    # persistent kernel must carry the FP64 one beside it.
    prob = W.amplitude(seed=1, n_integrals=6, n_sectors=24, d_lo=3, d_hi=7, m=8, n0=1009)
    if mixed:
        sec = prob.sectors[5]
        c0 = float(sec.f_coef[np.flatnonzero(sec.f_exp.sum(axis=1) == 0)[0]])
        i = int(np.flatnonzero(sec.f_exp.sum(axis=1) > 0)[0])
        sec.f_coef[i] = -0.5 * min(c0, float(sec.f_coef[i]))
    sizes, a_tab = ladder(seed=2)
    tau = np.array([float(s.d) for s in prob.sectors])
    out = {}
    for prec in (qmc.QMC_PREC_FP64, qmc.QMC_PREC_FP32):
        plan = qmc.Plan(prob, n_max=int(sizes[-1]), precision=prec)
        out[prec] = plan.amp_evaluate(prob.amp_coef, epsrel=5e-4, lattice_n=sizes,
                                      lattice_a=a_tab, tau=tau, n_presample=1009, mode=1)
        del plan
    v64, e64, n64, s64 = out[qmc.QMC_PREC_FP64]
    v32, e32, n32, s32 = out[qmc.QMC_PREC_FP32]
    assert s32["converged"] == 1 and s32["rounds"] == s64["rounds"]
    assert np.array_equal(n32, n64)
    scale = np.abs(v64) + np.abs(e64)
    dev = np.abs(v32 - v64) / scale
    print("mixed", mixed, "max rel deviation", dev.max(), flush=True)
    assert np.all(dev <= 1e-5)


@pytest.mark.parametrize("m", [3, 5])
def test_device_mode_fp32_with_odd_shift_count(qmc, m):
    # an odd number of shifts gives an odd shift tile while the FP32 batched form takes
    # two shifts per pass: the last pass of a tile has one live shift, whose partner slot
    # re-reads a shift inside the tile and is dropped.  Same rounds and lattices as the
    # FP64 batched form, sums within the FP32 bar.
    prob = W.amplitude(seed=1, n_integrals=6, n_sectors=24, d_lo=3, d_hi=6, m=m, n0=1009)
    sizes, a_tab = ladder(seed=2)
    tau = np.array([float(s.d) for s in prob.sectors])
    out = {}
    for prec in (qmc.QMC_PREC_FP64, qmc.QMC_PREC_FP32):
        plan = qmc.Plan(prob, n_max=int(sizes[-1]), precision=prec)
        assert plan.launch_shape()["shift_tile"] % 2 == 1
        out[prec] = plan.amp_evaluate(prob.amp_coef, epsrel=5e-4, lattice_n=sizes,
                                      lattice_a=a_tab, tau=tau, n_presample=1009, mode=1)
        del plan
    v64, e64, n64, s64 = out[qmc.QMC_PREC_FP64]
    v32, e32, n32, s32 = out[qmc.QMC_PREC_FP32]
    assert s32["rounds"] == s64["rounds"] and np.array_equal(n32, n64)
    dev = np.abs(v32 - v64) / (np.abs(v64) + np.abs(e64))
    print("m", m, "max rel deviation", dev.max(), flush=True)
    assert np.all(dev <= 1e-5)


@pytest.mark.parametrize("mode", [0, 1])
def test_timeout_returns_valid_partial_results(qmc, mode):
    # non-integer powers of U and F keep the lattice error well above 1e-15 on every rung,
    # so the target is out of reach (polynomial integrands, by contrast, can be integrated
    # to rounding level by the korobov-transformed rule and do converge there)
    prob = W.amplitude(seed=3, n_integrals=2, n_sectors=6, d_lo=3, d_hi=5, m=8, n0=1009)
    sizes, a_tab = ladder()
    plan = qmc.Plan(prob, n_max=int(sizes[-1]))
    val, err, nfin, st = plan.amp_evaluate(prob.amp_coef, epsrel=1e-15, lattice_n=sizes,
                                           lattice_a=a_tab, n_presample=1009, timeout_s=1e-9,
                                           mode=mode)
    assert st["converged"] == 0 and st["rounds"] >= 1
    # the host loop checks the limit every round; the batched form between queued batches
    # of rounds, so it may stop on the largest lattices before a check
    if mode == 0:
        assert st["status"] == -5 and st["timed_out"] == 1 and st["rounds"] == 1
    else:
        assert st["status"] in (0, -5) and st["timed_out"] == (st["status"] == -5)
    assert np.all(np.isfinite(val)) and np.all(np.abs(err) > 0)


@pytest.mark.parametrize("mode", [0, 1])
def test_rounding_level_target_on_polynomial_integrands(qmc, mode):
    # a target near the FP64 rounding level is reached where the integrands are smooth enough
    prob, exact = closed_form_problem()
    sizes, a_tab = ladder()
    val, err, nfin, st = _compare(qmc, prob, [[1.0, 1.0, 1.0]], sizes, a_tab, np.ones(6), 1e-15,
                                  1009, mode=mode)
    assert st["converged"] == 1
    assert np.all(np.abs(val[0] - exact.sum(axis=0)) <= 1e-13)


def test_invalid_amplitude_arguments(qmc):
    prob, _ = closed_form_problem()
    sizes, a_tab = ladder()
    plan = qmc.Plan(prob, n_max=int(sizes[-1]))
    with pytest.raises(qmc.QmcError, match="ascend"):
        plan.amp_evaluate([[1.0, 1.0, 1.0]], 1e-6, lattice_n=sizes[::-1].copy(),
                          lattice_a=a_tab[::-1].copy())
    with pytest.raises(qmc.QmcError, match="epsrel"):
        plan.amp_evaluate([[1.0, 1.0, 1.0]], 0.0, lattice_n=sizes, lattice_a=a_tab)
    with pytest.raises(qmc.QmcError, match="n_max"):
        plan.amp_evaluate([[1.0, 1.0, 1.0]], 1e-6, lattice_n=np.array([2**40 + 15], np.uint64),
                          lattice_a=np.ones((1, 8), np.uint64))


@pytest.mark.parametrize("mode", [0, 1])
def test_measured_costs_parity(qmc, mode):
    # tau measured while the loop runs (ticks per evaluation of every sector, Sec. 2.1.3):
    # the oracle's loop, given the costs each allocation used, takes the same rounds and
    # lattices and gives the same sums
    prob = W.amplitude(seed=1, n_integrals=6, n_sectors=24, d_lo=3, d_hi=6, m=8, n0=1009)
    sizes, a_tab = ladder(seed=2)
    coef = np.array([prob.amp_coef])
    plan = qmc.Plan(prob, n_max=int(sizes[-1]))
    val, err, nfin, st = plan.amp_evaluate(coef, epsrel=1e-5, lattice_n=sizes, lattice_a=a_tab,
                                           tau=None, n_presample=1009, mode=mode, return_tau=True)
    taus = st["tau_used"]
    print("rounds", st["rounds"], "converged", st["converged"], "tau rows", taus.shape, flush=True)
    # one row per allocation: after every round but a converged last one
    assert taus.shape[1] == len(prob.sectors)
    assert taus.shape[0] == st["rounds"] - (1 if st["converged"] else 0)
    assert np.all(taus > 0) and np.all(np.isfinite(taus))
    d = np.array([s.d for s in prob.sectors])
    # the cost per evaluation grows with the dimension (more monomials, more transforms)
    assert np.median(taus[0][d == d.max()]) > np.median(taus[0][d == d.min()])
    ov, oe, on, orounds, oconv = oracle.adaptive_amplitude(prob, coef, sizes, a_tab, taus,
                                                           epsrel=1e-5, n_presample=1009)
    assert st["rounds"] == orounds and bool(st["converged"]) == oconv
    assert np.array_equal(nfin, on)
    scale = np.abs(ov) + np.abs(oe)
    assert np.all(np.abs(val - ov) <= 1e-12 * scale)


def test_specialised_persistent_kernel_parity(qmc):
    # the batched form with its persistent kernel generated for the plan (the integrands
    # of every sector behind a switch): same rounds, lattices and sums as the oracle's loop
    prob = W.amplitude(seed=1, n_integrals=6, n_sectors=24, d_lo=3, d_hi=6, m=8, n0=1009)
    sizes, a_tab = ladder(seed=2)
    tau = np.array([float(s.d) for s in prob.sectors])
    coef = np.array([prob.amp_coef, prob.amp_coef * (0.5 - 1j)])
    _compare(qmc, prob, coef, sizes, a_tab, tau, 2e-6, 1009, persistent=True, mode=1)


def test_specialised_persistent_kernel_fp32(qmc):
    # FP32 batched form, specialised against table-driven on the same ladder and costs:
    # same rounds and final lattices, sums within the FP32 bar on their scale, and the
    # specialised form against the FP64 oracle loop within that bar too
    prob = W.amplitude(seed=1, n_integrals=6, n_sectors=24, d_lo=3, d_hi=7, m=8, n0=1009)
    sizes, a_tab = ladder(seed=2)
    tau = np.array([float(s.d) for s in prob.sectors])
    out = {}
    for spec in (False, True):
        plan = qmc.Plan(prob, n_max=int(sizes[-1]), precision=qmc.QMC_PREC_FP32)
        if spec:
            plan.specialize(persistent=True)
        out[spec] = plan.amp_evaluate(prob.amp_coef, epsrel=5e-4, lattice_n=sizes,
                                      lattice_a=a_tab, tau=tau, n_presample=1009, mode=1)
        del plan
    v0, e0, n0, s0 = out[False]
    v1, e1, n1, s1 = out[True]
    assert s1["converged"] == 1 and s1["rounds"] == s0["rounds"]
    assert np.array_equal(n1, n0)
    scale = np.abs(v0) + np.abs(e0)
    print("max deviation specialised vs table-driven", float((np.abs(v1 - v0) / scale).max()),
          flush=True)
    assert np.all(np.abs(v1 - v0) <= 1e-5 * scale)
    ov, oe, on, orounds, _ = oracle.adaptive_amplitude(prob, prob.amp_coef, sizes, a_tab, tau,
                                                       epsrel=5e-4, n_presample=1009)
    assert orounds == s1["rounds"] and np.array_equal(on, n1)
    assert np.all(np.abs(v1 - ov) <= 1e-5 * (np.abs(ov) + np.abs(oe)))


def test_specialised_persistent_kernel_follows_the_plan(qmc):
    # attaching a flow changes the plan's sectors without a flow: the specialised kernel no
    # longer matches and the batched form runs the library's own (same results as host mode)
    from oracle import flow as OF
    prob = W.amplitude(seed=1, n_integrals=6, n_sectors=24, d_lo=3, d_hi=6, m=8, n0=1009)
    sizes, a_tab = ladder(seed=2)
    tau = np.array([float(s.d) for s in prob.sectors])
    res = {}
    for mode in (0, 1):
        plan = qmc.Plan(prob, n_max=int(sizes[-1]))
        plan.specialize(persistent=True)
        d = prob.sectors[0].d
        plan.attach_flow(0, qmc.flow.Flow(d, params=OF.flatten(OF.init_params(d, seed=3))))
        res[mode] = plan.amp_evaluate(prob.amp_coef, epsrel=2e-6, lattice_n=sizes,
                                      lattice_a=a_tab, tau=tau, n_presample=1009, mode=mode)
        del plan
    (v0, e0, n0, s0), (v1, e1, n1, s1) = res[0], res[1]
    assert s0["rounds"] == s1["rounds"] and np.array_equal(n0, n1)
    assert np.all(np.abs(v1 - v0) <= 1e-12 * (np.abs(v0) + np.abs(e0)))
