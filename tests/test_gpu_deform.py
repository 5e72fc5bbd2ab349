"""GPU parity of the contour-deformed (complex) integrand with the oracle.

Per-shift complex sums are compared element by element with the oracle's on the same
lattices and shifts (relative 1e-12 of max(|Q|, (1/n) sum |W J f|)); sign-check counts
and the presample choice of the deformation parameter must be identical.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def qmc():
    import __graft_entry__ as g
    g._ensure_built()
    import torch
    import paper_2305_19768_amd as q
    torch.cuda.set_device(0)
    return q


def _mixed_sector(rng, d, n, lam, u_pow=1, f_pow2=-6, logc=None, x_pow2=None,
                  transform="korobov3", a=None):
    """Sector whose F has coefficients of both signs (F changes sign on the cube)."""
    u_exp, u_coef = W.random_polynomial(rng, d, int(rng.integers(3, 7)), 2)
    f_exp, _ = W.random_polynomial(rng, d, int(rng.integers(6, 16)), 3)
    f_coef = rng.uniform(-1.0, 1.0, size=len(f_exp))
    f_coef[0] = abs(f_coef[0]) + 0.05          # constant term of F positive
    if a is None:
        a = int(W._korobov_candidates(rng, n, 1)[0])
    return W.Sector(d=d, u_exp=u_exp, u_coef=u_coef, f_exp=f_exp, f_coef=f_coef,
                    x_pow2=np.zeros(d, np.int32) if x_pow2 is None else np.asarray(x_pow2, np.int32),
                    u_pow=u_pow, f_pow2=f_pow2,
                    logc=W.TWO_LOOP_LOGC.copy() if logc is None else np.asarray(logc, float),
                    n=n, a=a, transform=transform, deform_lambda=lam)


def _compare(qmc, prob, **plan_kw):
    plan = qmc.Plan(prob, **plan_kw)
    assert plan.complex
    q, mean, err = plan.integrate(check=False)
    q = q.cpu().numpy()
    viol = plan.sign_violations()
    worst = 0.0
    for s, sec in enumerate(prob.sectors):
        Q, S, ov, _ = oracle.sector_sums_deformed(sec, prob.shifts[s], threads=8)
        g = q[s, :, :, 0] + 1j * q[s, :, :, 1]
        scale = np.maximum(np.abs(Q), S)
        dev = np.abs(g - Q) / scale
        worst = max(worst, float(dev.max()))
        assert np.all(dev <= TOL), (s, float(dev.max()))
        assert int(viol[s]) == ov, (s, int(viol[s]), ov)
        # statistics of the real and imaginary parts
        mr, er = oracle.estimate(Q.real)
        mi, ei = oracle.estimate(Q.imag)
        mg = mean[s].cpu().numpy()
        eg = err[s].cpu().numpy()
        sc = np.max(S, axis=0)
        assert np.all(np.abs(mg[:, 0] - mr) <= TOL * sc) and np.all(np.abs(mg[:, 1] - mi) <= TOL * sc)
        assert np.allclose(eg[:, 0], er, rtol=1e-6, atol=TOL * np.max(sc))
        assert np.allclose(eg[:, 1], ei, rtol=1e-6, atol=TOL * np.max(sc))
    return plan, worst


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6, 7, 8])
def test_deformed_sector_parity_by_dimension(qmc, d):
    rng = np.random.default_rng(100 + d)
    secs, shifts = [], []
    for t in range(2):
        n = W.next_prime(1500 + 700 * t)
        sec = _mixed_sector(rng, d, n, lam=0.0)
        sh = W.uniform_shifts(rng, 8, d)
        sec.deform_lambda, _ = oracle.choose_lambda(sec, sh, 0.5, 509,
                                                    int(W._korobov_candidates(rng, 509, 1)[0]))
        secs.append(sec)
        shifts.append(sh)
    prob = W.Problem(sectors=secs, order_lo=-2, m=8, shifts=shifts)
    plan, worst = _compare(qmc, prob)
    print("d", d, "lambda", [s.deform_lambda for s in secs], "worst rel", worst, flush=True)


def test_deformed_integrand_features(qmc):
    # half-integer and negative x powers, negative U power, half-integer F power, four
    # orders with logs up to the cube, every transform family
    rng = np.random.default_rng(7)
    secs, shifts = [], []
    cases = [dict(x_pow2=[1, 0, -1], u_pow=-2, f_pow2=-3, transform="korobov3"),
             dict(x_pow2=[2, 3, 0], u_pow=0, f_pow2=1, transform="baker"),
             dict(x_pow2=[0, 0, 4], u_pow=2, f_pow2=-4, transform="korobov2"),
             dict(x_pow2=[-1, 1, 1], u_pow=-1, f_pow2=-2, transform="korobov5")]
    logc = [[1.0, 0.5, 0.0, 0.0], [0.0, -2.0, 1.0, 0.0], [0.3, 0.0, 0.0, 1.5],
            [0.0, 0.0, 0.0, 1.0]]
    for c in cases:
        sec = _mixed_sector(rng, 3, 2003, lam=0.25, logc=logc, **c)
        secs.append(sec)
        shifts.append(W.uniform_shifts(rng, 8, 3))
    prob = W.Problem(sectors=secs, order_lo=0, m=8, shifts=shifts)
    _compare(qmc, prob)


def test_real_and_deformed_sectors_in_one_plan(qmc):
    # lambda = 0 sectors of a complex plan run on the real contour with the F - i0 branch
    rng = np.random.default_rng(11)
    euc = W._two_loop_sector(rng, 4, 1009, 0)
    phys0 = _mixed_sector(rng, 3, 1013, lam=0.0)
    phys = _mixed_sector(rng, 5, 1019, lam=0.125)
    secs = [euc, phys0, phys]
    shifts = [W.uniform_shifts(rng, 16, s.d) for s in secs]
    prob = W.Problem(sectors=secs, order_lo=-2, m=16, shifts=shifts)
    plan, _ = _compare(qmc, prob)
    q, _, _ = plan.integrate(check=False)
    assert float(q[0, :, :, 1].abs().max()) == 0.0     # Euclidean, undeformed: real


def test_sign_check_counts_status_and_presample_choice(qmc):
    f = [(1.0, (0, 0)), (-6.0, (1, 0)), (6.0, (2, 0)), (-3.0, (1, 1)), (4.0, (3, 0)),
         (2.0, (0, 3))]
    rng = np.random.default_rng(0)
    secs = []
    for lam in (4.0, 1.0, 0.25):
        secs.append(W.custom_sector(2, [(1.0, (0, 0))], f, f_pow2=-2, transform="korobov3",
                                    n=1009, a=76, deform_lambda=lam))
    shifts = [W.uniform_shifts(rng, 4, 2) for _ in secs]
    prob = W.Problem(sectors=secs, order_lo=0, m=4, shifts=shifts)
    plan, _ = _compare(qmc, prob)
    viol = plan.sign_violations()
    assert viol[0] > 0 and viol[2] == 0
    with pytest.raises(qmc.QmcError) as ei:
        plan.check_status()
    assert ei.value.code == -6
    lam, halv, rc = plan.choose_deformation(1009, max_halvings=8)
    assert rc == 0
    for s, sec in enumerate(secs):
        ol, oh = oracle.choose_lambda(sec, shifts[s], sec.deform_lambda, 1009, 76,
                                      max_halvings=8)
        assert lam[s] == ol and halv[s] == oh, (s, lam[s], ol)
    plan.integrate()                       # chosen parameters: status clean
    assert not plan.sign_violations().any()
    # a budget of no halvings cannot fix the first sector
    plan.set_deformation([4.0, 1.0, 0.25])
    lam, halv, rc = plan.choose_deformation(1009, max_halvings=0)
    assert rc == -6 and lam[0] == 4.0 and halv[0] == 0


@pytest.mark.parametrize("kind", ["inverse", "log"])
def test_bubble_above_threshold_on_gpu(qmc, kind):
    s, m2 = 10.0, 1.0
    beta = math.sqrt(1 - 4 * m2 / s)
    f_terms = [(m2, (0,)), (-s, (1,)), (s, (2,))]
    if kind == "inverse":
        sec = W.custom_sector(1, [(1.0, (0,))], f_terms, f_pow2=-2, logc=[[1.0]],
                              transform="korobov3", n=1000003, deform_lambda=0.5)
        exact = 2 / (s * beta) * (math.log((1 - beta) / (1 + beta)) + 1j * math.pi)
    else:
        sec = W.custom_sector(1, [(1.0, (0,))], f_terms, logc=[[0.0, 1.0]],
                              transform="korobov3", n=1000003, deform_lambda=0.5)
        exact = (math.log(m2) - 2 + beta * math.log((1 + beta) / (1 - beta))
                 - 1j * math.pi * beta)
    rng = np.random.default_rng(1)
    prob = W.Problem(sectors=[sec], order_lo=0, m=16, shifts=[W.uniform_shifts(rng, 16, 1)])
    plan = qmc.Plan(prob)
    lam, _, rc = plan.choose_deformation(10007)
    assert rc == 0
    _, mean, err = plan.integrate()
    mean, err = mean.cpu().numpy()[0, 0], err.cpu().numpy()[0, 0]
    assert abs(mean[0] - exact.real) <= 6 * err[0] + 1e-12
    assert abs(mean[1] - exact.imag) <= 6 * err[1] + 1e-12
    assert err[0] < 1e-8 and err[1] < 1e-8


def test_physical_scan_sample_parity(qmc):
    prob = W.physical_scan(seed=1, n_points=3, n_sectors=5, d_lo=3, d_hi=8, n=2003, m=8)
    plan = qmc.Plan(prob)
    lam, _, rc = plan.choose_deformation(509)
    assert rc == 0
    for s, sec in enumerate(prob.sectors):
        sec.deform_lambda = float(lam[s])
    _compare(qmc, prob)


def test_complex_plan_rejected_by_amp_evaluate(qmc):
    rng = np.random.default_rng(3)
    sec = _mixed_sector(rng, 2, 1009, lam=0.25)
    prob = W.Problem(sectors=[sec], order_lo=-2, m=4, shifts=[W.uniform_shifts(rng, 4, 2)])
    plan = qmc.Plan(prob)
    with pytest.raises(qmc.QmcError, match="complex"):
        plan.amp_evaluate([[1.0]], 1e-3, lattice_n=np.array([1009], np.uint64),
                          lattice_a=np.ones((1, 8), np.uint64))


# ---------------------------------------------------------------- FP32 bulk form
# The gradient, Hessian, U(z) and F(z) in FP32; Jacobian, powers, logarithm and
# accumulation in FP64.  Sums against the FP64 oracle within TOL32 of the same scale;
# the worst relative deviation is printed per case.
TOL32 = 1e-5


def _compare32(qmc, prob, fp64_sectors=()):
    plan = qmc.Plan(prob, precision=qmc.QMC_PREC_FP32)
    assert plan.complex
    q, mean, err = plan.integrate(check=False)
    q, mean, err = q.cpu().numpy(), mean.cpu().numpy(), err.cpu().numpy()
    viol = plan.sign_violations()
    worst = 0.0
    for s, sec in enumerate(prob.sectors):
        Q, S, ov, _ = oracle.sector_sums_deformed(sec, prob.shifts[s], threads=8)
        g = q[s, :, :, 0] + 1j * q[s, :, :, 1]
        dev = np.abs(g - Q) / np.maximum(np.abs(Q), S)
        tol = TOL if s in fp64_sectors else TOL32
        assert np.all(dev <= tol), (s, float(dev.max()))
        # the stated error (shift error + the calibrated FP32 bound) covers the FP32
        # estimate's distance from the FP64 oracle's, part by part
        mo = Q.mean(axis=0)
        assert np.all(np.abs(mean[s, :, 0] - mo.real) <= err[s, :, 0]), s
        assert np.all(np.abs(mean[s, :, 1] - mo.imag) <= err[s, :, 1]), s
        if s not in fp64_sectors:
            worst = max(worst, float(dev.max()))
        # FP32 sign check: violations above FP32 rounding (2^-20 |F|) only, so counts
        # near the margin may differ from the FP64 oracle's
        assert abs(int(viol[s]) - ov) <= max(2, ov // 100), (s, int(viol[s]), ov)
    return plan, worst


@pytest.mark.parametrize("d", [1, 3, 5, 6, 8])
def test_deformed_fp32_bulk_parity_by_dimension(qmc, d):
    rng = np.random.default_rng(100 + d)
    secs, shifts = [], []
    for t in range(2):
        n = W.next_prime(1500 + 700 * t)
        sec = _mixed_sector(rng, d, n, lam=0.0)
        sh = W.uniform_shifts(rng, 8, d)
        sec.deform_lambda, _ = oracle.choose_lambda(sec, sh, 0.5, 509,
                                                    int(W._korobov_candidates(rng, 509, 1)[0]))
        assert sec.deform_lambda > 0
        secs.append(sec)
        shifts.append(sh)
    prob = W.Problem(sectors=secs, order_lo=-2, m=8, shifts=shifts)
    _, worst = _compare32(qmc, prob)
    print("d", d, "FP32 bulk worst rel. deviation", worst, flush=True)


def test_deformed_fp32_bulk_mixed_plan_and_scan(qmc):
    # Euclidean sector without cancellation: FP32 bulk; undeformed sector whose F changes
    # sign: stays FP64 (bit-level parity); deformed sector: FP32 bulk
    rng = np.random.default_rng(11)
    euc = W._two_loop_sector(rng, 4, 1009, 0)
    phys0 = _mixed_sector(rng, 3, 1013, lam=0.0)
    phys = _mixed_sector(rng, 5, 1019, lam=0.125)
    secs = [euc, phys0, phys]
    shifts = [W.uniform_shifts(rng, 16, s.d) for s in secs]
    prob = W.Problem(sectors=secs, order_lo=-2, m=16, shifts=shifts)
    _, worst = _compare32(qmc, prob, fp64_sectors=(1,))
    print("mixed plan FP32 bulk worst rel. deviation", worst, flush=True)
    scan = W.physical_scan(seed=1, n_points=3, n_sectors=5, d_lo=3, d_hi=8, n=2003, m=8)
    plan = qmc.Plan(scan)
    lam, _, rc = plan.choose_deformation(509)
    assert rc == 0
    for s, sec in enumerate(scan.sectors):
        sec.deform_lambda = float(lam[s])
    _, worst = _compare32(qmc, scan)
    print("scan FP32 bulk worst rel. deviation", worst, flush=True)


def test_bubble_above_threshold_fp32_bulk(qmc):
    s, m2 = 10.0, 1.0
    beta = math.sqrt(1 - 4 * m2 / s)
    f_terms = [(m2, (0,)), (-s, (1,)), (s, (2,))]
    sec = W.custom_sector(1, [(1.0, (0,))], f_terms, logc=[[0.0, 1.0]],
                          transform="korobov3", n=1000003, deform_lambda=0.5)
    exact = (math.log(m2) - 2 + beta * math.log((1 + beta) / (1 - beta))
             - 1j * math.pi * beta)
    rng = np.random.default_rng(1)
    prob = W.Problem(sectors=[sec], order_lo=0, m=16, shifts=[W.uniform_shifts(rng, 16, 1)])
    plan = qmc.Plan(prob, precision=qmc.QMC_PREC_FP32)
    lam, _, rc = plan.choose_deformation(10007)
    assert rc == 0
    _, mean, err = plan.integrate()
    mean = mean.cpu().numpy()[0, 0]
    print("bubble FP32 bulk", mean, exact, flush=True)
    assert abs(mean[0] - exact.real) <= 1e-5 * abs(exact)
    assert abs(mean[1] - exact.imag) <= 1e-5 * abs(exact)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_integrate_deformed_equals_choice_then_integration(qmc, precision):
    """qmc_integrate_deformed (integrate, then re-integrate the sectors with a violating
    sample with lambda halved) gives what the full-lattice choice followed by an
    integration gives, after the presample choice of the deformation parameters: the same
    parameters, bit for bit the same sums for the sectors integrated once, and for the
    re-integrated ones (a launch over fewer sectors splits their lattices into other
    chunks, so the compensated sums may round differently) the same to 1e-13."""
    prob = W.physical_scan(seed=0, n_points=2)
    prec = qmc.QMC_PREC_FP32 if precision == "fp32" else qmc.QMC_PREC_FP64
    ref = qmc.Plan(prob, precision=prec)
    lam0, _, rc0 = ref.choose_deformation(4099)
    assert rc0 == 0
    lam_ref, halv_ref, rc_ref = ref.choose_deformation(prob.sectors[0].n)
    q_ref, m_ref, e_ref = ref.integrate(check=False)
    new = qmc.Plan(prob, precision=prec)
    new.set_deformation(lam0)
    q, m, e, lam, halv, rc = new.integrate_deformed()
    print("sectors halved on the full lattice", int(np.count_nonzero(halv)), flush=True)
    assert np.count_nonzero(halv) > 0          # the fallback was exercised
    assert rc == rc_ref == 0
    assert np.array_equal(lam, lam_ref) and np.array_equal(halv, halv_ref)
    once = halv == 0
    q, m, e = q.cpu().numpy(), m.cpu().numpy(), e.cpu().numpy()
    q_ref, m_ref, e_ref = q_ref.cpu().numpy(), m_ref.cpu().numpy(), e_ref.cpu().numpy()
    for a_, b_ in ((q, q_ref), (m, m_ref), (e, e_ref)):
        assert np.array_equal(a_[once].view(np.uint64), b_[once].view(np.uint64))
    # on the scale of each sector's largest sum (a real or imaginary part can be ~0; an
    # error is a spread of the shift sums)
    sq = np.abs(q_ref[~once]).max(axis=(1, 2, 3))[:, None, None, None]
    sm = np.abs(m_ref[~once]).max(axis=(1, 2))[:, None, None]
    print("re-integrated sectors: max |dq| / scale",
          float((np.abs(q[~once] - q_ref[~once]) / sq).max()), flush=True)
    assert np.all(np.abs(q[~once] - q_ref[~once]) <= 1e-13 * sq)
    assert np.all(np.abs(m[~once] - m_ref[~once]) <= 1e-13 * sm)
    assert np.all(np.abs(e[~once] - e_ref[~once]) <= 1e-13 * sm)
    # no sample of the final contours violates the sign check
    new.integrate(check=False)
    assert not np.any(new.sign_violations())


def test_integrate_deformed_without_halvings_reports_the_violation(qmc):
    """max_halvings = 0: one integration at the given parameters, the violation reported
    as QMC_E_SIGNCHECK with every output written (equal to a plain integration)."""
    prob = W.physical_scan(seed=0, n_points=2)
    plan = qmc.Plan(prob)
    lam0, _, _ = plan.choose_deformation(4099)
    q0, m0, e0 = plan.integrate(check=False)
    q0 = q0.cpu().numpy()
    viol = plan.sign_violations()
    assert np.any(viol)
    q, m, e, lam, halv, rc = plan.integrate_deformed(max_halvings=0)
    assert rc == -6   # QMC_E_SIGNCHECK
    assert np.array_equal(lam, lam0) and not np.any(halv)
    assert np.array_equal(q.cpu().numpy().view(np.uint64), q0.view(np.uint64))
