"""GPU parity of the plan-specialised (run-time generated and compiled) integrand kernels
against the CPU oracle, through the C ABI (qmc_specialize, then qmc_integrate).

Bars as in test_gpu_parity: per-shift sums within 1e-12 (FP64) or 1e-5 (FP32 integrand
form) of max(|Q_oracle|, (1/n) sum |W f|).  Also: the specialised and table-driven
kernels agree on the same plan; a launch shape the kernels were not compiled for, and a
sector that joins a class after specialisation, run on the table-driven kernels.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import flow as OF

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


def _check(q_gpu, prob, tol, sectors=None, shift_range=None):
    for s in (range(len(prob.sectors)) if sectors is None else sectors):
        sec = prob.sectors[s]
        kw = {} if shift_range is None else {"shift_range": shift_range}
        Qo, So = oracle.sector_sums(sec, prob.shifts[s], threads=8, **kw)
        got = q_gpu[s] if shift_range is None else q_gpu[s, shift_range[0]:shift_range[1]]
        rel = np.abs(got - Qo) / np.maximum(np.abs(Qo), So)
        print(f"sector {s}: d={sec.d} n={sec.n} max rel {rel.max():.2e}", flush=True)
        assert rel.max() <= tol, (s, rel.max())


@pytest.mark.parametrize("precision,tol", [("fp64", TOL), ("fp32", 1e-5)])
def test_specialized_two_loop_parity(qmc, precision, tol):
    prob = W.two_loop_integral(seed=0, n_scale=0.01)   # 40 sectors, d 4..6, n in [1e3, 1e5]
    prec = qmc.QMC_PREC_FP32 if precision == "fp32" else qmc.QMC_PREC_FP64
    plan = qmc.Plan(prob, precision=prec)
    sec_s = plan.specialize()
    print(f"specialised in {sec_s:.2f} s", flush=True)
    q, mean, err = plan.integrate()
    _check(q.cpu().numpy(), prob, tol)


def test_fp32_specialised_at_four_shifts_per_pass(qmc):
    prob = W.two_loop_integral(seed=0, n_scale=0.01)
    out = {}
    for spp in (2, 4):
        plan = qmc.Plan(prob, precision=qmc.QMC_PREC_FP32, shifts_per_pass=spp)
        plan.specialize()
        assert plan.launch_shape()["shifts_per_pass"] == spp
        out[spp] = plan.integrate()[0].cpu().numpy()
    _check(out[4], prob, 1e-5)
    # each shift's sum is formed by the same operations at either pass width
    print("max |spp4 - spp2|", np.max(np.abs(out[4] - out[2])), flush=True)
    assert np.array_equal(out[2], out[4])


@pytest.mark.parametrize("d,K,M,u_pow,f_pow2", [(1, 1, 0, 0, -2), (3, 2, 1, -1, -4), (5, 3, 2, 2, -6),
                                                (7, 4, 3, 1, -8), (8, 4, 1, 0, 4), (6, 3, 0, 3, 0)])
def test_specialized_fast_path_shapes(qmc, d, K, M, u_pow, f_pow2):
    rng = np.random.default_rng(7 * d + K)
    ue, uc = W.random_polynomial(rng, d, 6, 2)
    fe, fc = W.random_polynomial(rng, d, 15, 3)
    sec = W.Sector(d=d, u_exp=ue, u_coef=uc, f_exp=fe, f_coef=fc,
                   x_pow2=np.zeros(d, np.int32), u_pow=u_pow, f_pow2=f_pow2,
                   logc=rng.uniform(-1, 1, size=(K, M + 1)), n=20011,
                   a=int(rng.integers(2, 20009)), transform="korobov3")
    prob = W.single_problem(sec, m=8, seed=d)
    for spp in (1, 2, 4):
        plan = qmc.Plan(prob, shifts_per_pass=spp)
        plan.specialize()
        print(f"d={d} K={K} spp={spp}", flush=True)
        _check(plan.integrate()[0].cpu().numpy(), prob, TOL)


@pytest.mark.parametrize("transform", ["none", "baker", "korobov2", "korobov3", "korobov5"])
@pytest.mark.parametrize("x_pow2,u_pow,f_pow2", [([1, 0, 3], -2, -3), ([-3, 4, 1], 0, -1),
                                                 ([0, 2, 0], 1, 3)])
def test_specialized_generic_shapes(qmc, transform, x_pow2, u_pow, f_pow2):
    # integer and half-integer powers of x_j and F, every transform family, a log
    # polynomial of degree above K - 1: the specialised kernel against the oracle at one,
    # two and four shifts per pass
    sec = W.custom_sector(3, [(1.0, (0, 0, 0)), (0.5, (1, 0, 0)), (0.25, (0, 1, 1))],
                          [(0.3, (0, 0, 0)), (0.7, (1, 1, 0)), (0.2, (0, 0, 2)), (0.4, (1, 0, 1))],
                          x_pow2=x_pow2, u_pow=u_pow, f_pow2=f_pow2,
                          logc=[[1, 0, 0.5], [0.5, -1, 0]], n=20011, a=5467, transform=transform)
    prob = W.single_problem(sec, m=8, seed=1)
    for spp in (1, 2, 4):
        plan = qmc.Plan(prob, shifts_per_pass=spp)
        plan.specialize()
        print(f"{transform} x_pow2={x_pow2} spp={spp}", flush=True)
        _check(plan.integrate()[0].cpu().numpy(), prob, TOL)


def test_one_loop_sector_specialised(qmc):
    prob = W.one_loop_sector(seed=0, n=65521, m=16)
    plan = qmc.Plan(prob)
    q0 = plan.integrate()[0].cpu().numpy()
    plan.specialize()
    q1 = plan.integrate()[0].cpu().numpy()
    assert np.allclose(q1, q0, rtol=1e-12, atol=0.0)
    _check(q1, prob, TOL)


def test_specialized_agrees_with_table_driven(qmc):
    prob = W.two_loop_integral(seed=7, n_sectors=12, n_scale=0.02)
    plan = qmc.Plan(prob)
    q0 = plan.integrate()[0].cpu().numpy()
    plan.specialize()
    q1 = plan.integrate()[0].cpu().numpy()
    q2 = plan.integrate()[0].cpu().numpy()
    assert np.array_equal(q1, q2)                        # run-to-run bitwise
    assert np.allclose(q1, q0, rtol=1e-12, atol=0.0)     # same sums up to rounding order
    plan.specialize(off=True)
    assert np.array_equal(plan.integrate()[0].cpu().numpy(), q0)


def test_unspecialised_shape_and_class_fall_back(qmc):
    prob = W.two_loop_integral(seed=8, n_sectors=6, n_scale=0.01, m=8)
    plan = qmc.Plan(prob)
    # a flow on sector 0 at specialisation time: its class kernel has no case for it
    fl = qmc.flow.Flow(prob.sectors[0].d, params=OF.flatten(OF.init_params(prob.sectors[0].d, seed=3)))
    plan.attach_flow(0, fl)
    plan.specialize()
    plan.attach_flow(0, None)        # sector 0 rejoins its class: table-driven for that class
    _check(plan.integrate()[0].cpu().numpy(), prob, TOL)
    plan.set_launch_shape(256, 8, 1)  # compiled for two shifts per pass: table-driven
    _check(plan.integrate()[0].cpu().numpy(), prob, TOL)
    plan.specialize()                # now compiled for one shift per pass as well
    _check(plan.integrate()[0].cpu().numpy(), prob, TOL)


@pytest.mark.parametrize("precision,tol,shape", [("fp64", TOL, (256, 4, 4, 16384)),
                                                 ("fp64", TOL, (256, 8, 4, 8192)),
                                                 ("fp32", 1e-5, (256, 4, 2, 16384)),
                                                 ("fp32", 1e-5, (256, 2, 2, 32768))])
def test_specialized_largest_sector_full_size(qmc, precision, tol, shape):
    # the launch shapes the autotuner picks for the benchmark's FP64 and FP32 plans
    prob = W.two_loop_integral(seed=0)
    prec = qmc.QMC_PREC_FP32 if precision == "fp32" else qmc.QMC_PREC_FP64
    plan = qmc.Plan(prob, precision=prec)
    a = [plan.korobov_search(s.n, s.d, [int(c) for c in s.a_candidates])[0] for s in prob.sectors]
    plan.set_launch_shape(*shape)
    plan.specialize()
    q = plan.integrate(a=a)[0].cpu().numpy()
    assert np.all(np.isfinite(q))
    # the largest sector of every dimension class (one kernel each), on two shifts
    for d in sorted({sec.d for sec in prob.sectors}):
        s = max((i for i, sec in enumerate(prob.sectors) if sec.d == d),
                key=lambda i: prob.sectors[i].n)
        sec = dataclasses.replace(prob.sectors[s], a=int(a[s]))
        one = dataclasses.replace(prob, sectors=[sec], shifts=[prob.shifts[s]])
        _check(q[s:s + 1], one, tol, shift_range=(0, 2))
