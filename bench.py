"""Benchmark: integrand evaluations per second of randomized rank-1 lattice QMC on MI355X.

Workload (one step = one pass of the whole hot path over it): the two-loop-like
synthetic integral -- 40 sectors, d uniform in 4..6, U with 4-8 and F with 10-30
monomials, epsilon orders -2..0 with log^m F (m <= 2), per-sector prime lattice sizes
log-uniform in [1e5, 1e7], 32 random shifts -- integrated in FP64: lattice points,
korobov3 transform, integrand, compensated per-shift sums, shift means and errors.
One evaluation = one (lattice point, shift) sample of one sector, all orders.

Prints one JSON line.  `roofline` reports the integrand kernel against the FP64 vector
peak (the path is ALU-bound; it reads no per-sample data from memory): algorithmic
flops per launch (convention in `algorithmic_flops`) over the kernel time measured
with HIP events on the launch stream.  `cpu_baseline` times the CPU oracle on a
bounded sample of the same workload (every sector, one shift).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X: 256 CUs x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3    # MI355X published FP32 vector peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "qmc_gen_class_kernels_two_loop_traffic.json")

# The paper's own figures, quoted with their hardware as context (not a target: they are
# end-to-end wall times to a requested relative accuracy on the paper's integrals, which
# are not available here; the paper gives no evaluation rates, flop rates or FP32 results).
PAPER_FIGURES = {
    "hardware": {"gpu": "NVIDIA A100 80G, integrands compiled with CUDA 11.8.89",
                 "cpu": "AMD EPYC 7F32, 16 cores (32 threads), GCC 12.2.1 -O3 -mavx2 -mfma"},
    "kind": "wall time to the requested relative accuracy, all eps orders (seconds)",
    "hexatriangle (2-loop 5-point, section 3.1.4, table of its timings)": {
        "1e-4": {"gpu_disteval": 6.3, "gpu_intlib_qmc": 32.6, "cpu_disteval": 14.0},
        "1e-6": {"gpu_disteval": 90.0, "gpu_intlib_qmc": 402.0, "cpu_disteval": 498.0}},
    "pentabox_offshell (2-loop 5-point, section 3.1.5, table of its timings)": {
        "1e-4": {"gpu_disteval": 474.0, "gpu_intlib_qmc": 2934.0, "cpu_disteval": 2580.0}},
    "elliptic2L_physical (section 2.2, median-rule table; GPU, Disteval)": {
        "1e-8": {"cbc_lattices": 452.0, "median_r11": 37.0}},
}


def algorithmic_flops(sec, m: int) -> float:
    """Algorithmic flops of one evaluation of a sector (what the method computes, not
    what the kernel executes).  Convention: add, multiply = 1; FMA = 2; division, square
    root and log = 1 each.  Per evaluation:
      lattice    d adds (q + Delta) and d divisions k/n shared by the m shifts;
      korobov3   14 per coordinate (y(1-y), its cube, the factor 140, a 3-FMA Horner,
                 y^4 and the product), plus d-1 for W; baker 3, none 0;
      U, F       per monomial of total degree g: g multiplications by variables, one by
                 the coefficient, one add;
      base       one multiplication per unit of |integer exponent| of U and F and of x_j,
                 one square root if a half-integer exponent occurs, one division if a
                 negative exponent occurs;
      log F      1 if any order uses it;
      orders     per order: 2 max_log (Horner in log F) + 1 (base times polynomial) +
                 1 (weight) + 1 (accumulate).
    """
    import numpy as np
    d = sec.d
    f = d + d / m
    if sec.transform.startswith("korobov"):
        f += 14 * d + (d - 1)
    elif sec.transform == "baker":
        f += 3 * d
    for e in (np.asarray(sec.u_exp), np.asarray(sec.f_exp)):
        g = e.reshape(len(e), d).sum(axis=1)
        f += float(np.sum(g + 2))
    xp = np.asarray(sec.x_pow2)
    f += abs(int(sec.u_pow)) + abs(int(sec.f_pow2)) // 2 + int(np.sum(np.abs(xp) // 2))
    if (xp % 2).any() or sec.f_pow2 % 2:
        f += 1
    if sec.u_pow < 0 or sec.f_pow2 < 0 or (xp < 0).any():
        f += 1
    M = sec.M
    if M > 0:
        f += 1
    f += sec.K * (2 * M + 3)
    return f


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("qmc_kernels.hip", "qmc_device.h", "qmc_internal.h", "qmc_gen.cpp"):
        with open(os.path.join(ROOT, "paper_2305_19768_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(problem, threads: int):
    """CPU oracle on every sector with one shift (a bounded sample of the workload)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    from oracle import build as ob
    if not os.path.exists(ob.LIB):
        ob.build()
    order = sorted(range(len(problem.sectors)), key=lambda s: -problem.sectors[s].n)

    def run(s):
        oracle.sector_sums(problem.sectors[s], problem.shifts[s], shift_range=(0, 1))

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, order))
    dt = time.perf_counter() - t0
    evals = int(sum(s.n for s in problem.sectors))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": evals / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"all {len(problem.sectors)} sectors x 1 of {problem.m} shifts "
                      f"({evals} evaluations, FP64 scalar C, {dt:.1f} s)",
            "cpu_model": model, "host_cpus": os.cpu_count()}


def amplitude_leg(qmc, torch, repeats: int):
    """Wall time to a relative error of 1e-4 on every epsilon order of the synthetic
    amplitude (20 integrals, 500 sectors, d 3..7, 32 shifts, FP64 oracle-pinned method),
    for the plain FP64 host loop and the batched on-device forms in FP64 and FP32.  The
    lattice table (prime sizes, P_2-chosen Korobov parameters) is built once beforehand,
    as a precomputed table would be, and each form's launch shape is chosen by the
    autotuner on the presampling lattices; each timed call starts from the presampling
    round."""
    import numpy as np
    import workloads
    prob = workloads.amplitude(seed=0)
    sizes, cands = workloads.lattice_ladder(n_min=10007, n_max=1 << 26, ratio=1.5, n_cand=8)
    t0 = time.perf_counter()
    table = qmc.Plan(prob, n_max=int(sizes[-1])).lattice_table(sizes, cands)
    setup_s = time.perf_counter() - t0
    forms = {"fp64_host": (qmc.QMC_PREC_FP64, qmc.QMC_AMP_HOST),
             "fp64_device": (qmc.QMC_PREC_FP64, qmc.QMC_AMP_DEVICE),
             "fp32_device": (qmc.QMC_PREC_FP32, qmc.QMC_AMP_DEVICE)}
    out = {"workload": "amplitude: 20 integrals, 500 sectors, d 3..7, 32 shifts, orders "
                       "eps^-2..eps^0, korobov3, target epsrel 1e-4 per order",
           "lattice_sizes": [int(sizes[0]), int(sizes[-1]), len(sizes)],
           "table_setup_s": setup_s}
    vals = {}
    # launch shape of each form from the autotuner, timed on the presampling lattices
    l0 = int(np.searchsorted(sizes, 10007))
    n_tune = [int(sizes[l0])] * len(prob.sectors)
    a_tune = [int(table[l0, s.d - 1]) for s in prob.sectors]
    for name, (prec, mode) in forms.items():
        plan = qmc.Plan(prob, precision=prec, n_max=int(sizes[-1]))
        # the FP32 batched form runs its persistent kernel generated for the plan (one
        # program holding every sector's integrand; compiled once beforehand, as the
        # paper's integrand libraries are); the FP64 one keeps the library's (its
        # generated kernel takes minutes to compile for 500 sectors)
        spec_s = plan.specialize(persistent=True) if name == "fp32_device" else None
        shape = plan.autotune(n=n_tune, a=a_tune, reps=3, use_cache=False)
        times = []
        for _ in range(repeats + 1):              # first call warms up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            val, err, nfin, st = plan.amp_evaluate(prob.amp_coef, epsrel=1e-4, lattice_n=sizes,
                                                   lattice_a=table, n_presample=10007,
                                                   mode=mode)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
        rel = np.abs(err[0]) / np.abs(val[0])
        vals[name] = (val[0], err[0])
        out[name] = {"wall_s": float(np.median(times[1:])), "rounds": st["rounds"],
                     "converged": st["converged"], "evaluations": st["evaluations"],
                     "max_rel_err": float(np.max(rel)), "max_n": int(np.max(nfin)),
                     "launch": {k: shape[k] for k in ("block", "shift_tile", "shifts_per_pass")},
                     "specialised_persistent_kernel_compile_s": spec_s}
        print(f"# amplitude {name}: {out[name]}", file=sys.stderr, flush=True)
        del plan
    out["fp32_flow"] = amplitude_flow_form(qmc, torch, prob, sizes, table)
    v64, e64 = vals["fp64_host"]
    for name in ("fp64_device", "fp32_device"):
        v, e = vals[name]
        # distance from the FP64 host-loop result in units of the combined error estimates
        out[name]["dev_vs_fp64_in_sigma"] = float(np.max(np.abs(v - v64) /
                                                         (np.abs(e) + np.abs(e64))))
    out["speedup_fp32_device_vs_fp64_host"] = (out["fp64_host"]["wall_s"] /
                                              out["fp32_device"]["wall_s"])
    return out


def train_flows(torch, jobs, n_streams: int = 4):
    """Trains the flows of jobs [(flow, x, w, train keyword arguments)] on n_streams
    streams at once (default priority, one host thread each): one flow's minibatches
    fill only a fraction of the GPU.  The inputs were made on the current stream, which
    the streams wait for; returns when every flow is trained."""
    from concurrent.futures import ThreadPoolExecutor
    main = torch.cuda.current_stream()
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    for st in streams:
        st.wait_stream(main)

    def work(i):
        with torch.cuda.stream(streams[i]):
            for k in range(i, len(jobs), n_streams):
                fl, x, w, kw = jobs[k]
                fl.train(x, w, **kw)
        streams[i].synchronize()

    with ThreadPoolExecutor(max_workers=n_streams) as ex:
        list(ex.map(work, range(n_streams)))
    for st in streams:
        main.wait_stream(st)


def flow_training_seconds(qmc, torch, d: int, samples: int, batches: int, epochs: int) -> float:
    """Wall time to train one flow of dimension d on `samples` samples (batches x epochs
    Adam steps), from one timed epoch of a fresh flow on random samples (a property of
    the network and the GPU, measured once beforehand like a launch shape)."""
    x = torch.rand((samples, d), dtype=torch.float64, device="cuda") * 0.98 + 0.01
    w = torch.rand(samples, dtype=torch.float64, device="cuda") + 0.5
    fl = qmc.flow.Flow(d, seed=1)
    fl.train(x, w, batches=batches, epochs=1, lr=2e-3)     # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fl.train(x, w, batches=batches, epochs=1, lr=2e-3)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * epochs


def amplitude_flow_form(qmc, torch, prob, sizes, table, n_tr: int = 262144,
                        batches: int = 16, epochs: int = 3):
    """The batched FP32 form with learned transforms, everything from the first
    presample on inside the timed region.  The amplitude is evaluated in the batched FP32
    form with costs measured on the device; a flow can save at most its sector's share of
    that evaluation's wall time (its measured ticks over all ticks), so a flow is trained
    only for sectors whose share exceeds the time to train one (measured beforehand per
    dimension).  Trained flows are kept where the square root of the variance ratio at
    the sector's final lattice exceeds the cost ratio per evaluation (the work to equal
    error under the n^-2 decay the allocation assumes), and the amplitude is evaluated
    again with them; with no candidate, the first evaluation is the result."""
    import dataclasses
    import numpy as np
    import workloads
    dims = sorted({s.d for s in prob.sectors})
    t_train = {d: flow_training_seconds(qmc, torch, d, n_tr, batches, epochs) for d in dims}
    plan = qmc.Plan(prob, precision=qmc.QMC_PREC_FP32, n_max=int(sizes[-1]))
    plan.specialize(persistent=True)   # compiled by the FP32 leg already: a cache hit
    # the batched FP32 form's launch shape (cached from its own leg), outside the timing
    plan.autotune(n=[int(sizes[0])] * len(prob.sectors),
                  a=[int(table[0, s.d - 1]) for s in prob.sectors], reps=3, use_cache=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    val, err, nfin, st = plan.amp_evaluate(prob.amp_coef, epsrel=1e-4, lattice_n=sizes,
                                           lattice_a=table, n_presample=10007,
                                           mode=qmc.QMC_AMP_DEVICE, return_tau=True)
    torch.cuda.synchronize()
    t_eval = time.perf_counter() - t0
    # each sector's ticks over the rounds: tau (ticks per evaluation) of the last
    # allocation times the evaluations at its final lattice (its largest share)
    tau = st["tau_used"][-1] if len(st["tau_used"]) else np.ones(len(prob.sectors))
    ticks = tau * nfin.astype(np.float64) * prob.m
    share_s = t_eval * ticks / ticks.sum()
    cand = [s for s in range(len(prob.sectors)) if share_s[s] > t_train[prob.sectors[s].d]]
    out = {"candidates": len(cand), "largest_sector_share_ms": float(share_s.max() * 1e3),
           "training_ms_per_flow": {str(d): float(t * 1e3) for d, t in t_train.items()},
           "first_evaluation_s": t_eval}
    kept = []
    if cand:
        l_tr = int(np.searchsorted(sizes, n_tr))
        sub = workloads.Problem(sectors=[dataclasses.replace(prob.sectors[s], integral=0)
                                         for s in cand], order_lo=prob.order_lo, m=prob.m,
                                shifts=[prob.shifts[s] for s in cand])
        psub = qmc.Plan(sub, precision=qmc.QMC_PREC_FP32, n_max=int(sizes[-1]))
        flows, jobs = [], []
        for k, s in enumerate(cand):
            d = prob.sectors[s].d
            x, w = psub.flow_samples(k, int(sizes[l_tr]), int(table[l_tr, d - 1]), shift=0)
            fl = qmc.flow.Flow(d, seed=s)
            jobs.append((fl, x, w, {"batches": batches, "epochs": epochs, "lr": 2e-3}))
            flows.append(fl)
        train_flows(torch, jobs)
        n_fin = [int(nfin[s]) for s in cand]
        a_fin = [int(table[int(np.searchsorted(sizes, n)), prob.sectors[s].d - 1])
                 for s, n in zip(cand, n_fin)]
        psub.enable_timing(True)
        _, _, e0 = psub.integrate(n=n_fin, a=a_fin)
        k_plain, _ = psub.read_timing()
        for k, fl in enumerate(flows):
            psub.attach_flow(k, fl)
        psub.enable_timing(True)
        _, _, e1 = psub.integrate(n=n_fin, a=a_fin)
        k_flow, _ = psub.read_timing()
        ratio = (e0.cpu().numpy() ** 2).sum(axis=1) / (e1.cpu().numpy() ** 2).sum(axis=1)
        cost_ratio = k_flow / k_plain
        kept = [k for k in range(len(cand)) if np.sqrt(ratio[k]) > cost_ratio]
        out.update({"variance_ratio_plain_over_flow": [float(r) for r in ratio],
                    "cost_ratio_flow_over_plain": float(cost_ratio)})
        if kept:
            for k in kept:
                plan.attach_flow(cand[k], flows[k])
            val, err, nfin, st = plan.amp_evaluate(prob.amp_coef, epsrel=1e-4,
                                                   lattice_n=sizes, lattice_a=table,
                                                   n_presample=10007, mode=qmc.QMC_AMP_DEVICE)
    torch.cuda.synchronize()
    rel = np.abs(err[0]) / np.abs(val[0])
    out.update({"flows_trained": len(cand), "flows_kept": len(kept),
                "wall_s": time.perf_counter() - t0, "rounds": st["rounds"],
                "converged": st["converged"], "max_rel_err": float(np.max(rel))})
    return out


def scan_leg(qmc, torch, n_points: int, steps: int):
    """Physical-region scan on the deformed contour (complex FP64): n_points kinematic
    points x 200 base sectors (d 3..8), n = 65521, 16 shifts, lambda chosen from
    presamples (n = 4099) by halving from 0.5, then halved again for the sectors that still
    violate the sign check on the full lattice (the fallback).  Reports complex
    evaluations per second of the integration step and how many sectors needed a
    smaller lambda in each pass."""
    import numpy as np
    import workloads
    prob = workloads.physical_scan(seed=0, n_points=n_points)
    plan = qmc.Plan(prob)
    t0 = time.perf_counter()
    lam, halv, rc = plan.choose_deformation(4099)
    # fallback: sectors still violating the sign check on the full lattice are halved again
    lam2, halv2, rc2 = plan.choose_deformation(65521)
    torch.cuda.synchronize()
    choose_s = time.perf_counter() - t0
    S, m, K = plan.S, plan.m, plan.K
    out = (torch.empty((S, m, K, 2), dtype=torch.float64, device="cuda"),
           torch.empty((S, K, 2), dtype=torch.float64, device="cuda"),
           torch.empty((S, K, 2), dtype=torch.float64, device="cuda"))
    plan.integrate(out=out, check=False)
    torch.cuda.synchronize()
    plan.enable_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.integrate(out=out, check=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kernel_ms, launches = plan.read_timing()
    plan.enable_timing(False)
    viol = plan.sign_violations()
    evals = prob.evals()
    m64 = out[1].cpu().numpy().copy()
    e64 = out[2].cpu().numpy().copy()
    # the same scan in two calls on a fresh plan: the presample choice, then the
    # integration with the sign-check fallback built in (qmc_integrate_deformed), which
    # integrates the sectors that need no further halving once
    del plan
    plan_w = qmc.Plan(prob)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan_w.choose_deformation(4099)
    _, mw, _, lamw, halvw, rcw = plan_w.integrate_deformed(out=out)
    torch.cuda.synchronize()
    workflow_s = time.perf_counter() - t0
    mw = mw.cpu().numpy()
    workflow = {"choice_then_integration_s": choose_s + el / steps,
                "presample_then_integrate_deformed_s": workflow_s,
                "same_lambda": bool(np.array_equal(lamw, lam2)),
                "max_rel_diff_of_estimates": float(np.max(
                    np.abs((mw[..., 0] - m64[..., 0]) + 1j * (mw[..., 1] - m64[..., 1])) /
                    np.maximum(np.hypot(m64[..., 0], m64[..., 1]), 1e-300)))}
    del plan_w
    # FP32 bulk (gradient, Hessian, U(z), F(z) in FP32; Jacobian, log, powers and sums in
    # FP64) with the same deformation parameters
    plan32 = qmc.Plan(prob, precision=qmc.QMC_PREC_FP32)
    plan32.set_deformation(lam2)
    plan32.integrate(out=out, check=False)
    torch.cuda.synchronize()
    plan32.enable_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan32.integrate(out=out, check=False)
    torch.cuda.synchronize()
    el32 = time.perf_counter() - t0
    k32, l32 = plan32.read_timing()
    plan32.enable_timing(False)
    viol32 = plan32.sign_violations()
    m32 = out[1].cpu().numpy()
    e32 = out[2].cpu().numpy()   # stated error: shift error + the FP32 rounding bound
    c64 = m64[..., 0] + 1j * m64[..., 1]
    c32 = m32[..., 0] + 1j * m32[..., 1]
    err = np.hypot(e64[..., 0], e64[..., 1])
    dev = np.abs(c32 - c64)
    rel = dev / np.maximum(np.abs(c64), 1e-300)
    del plan32
    return {"workload": f"physical_scan: {n_points} kinematic points x 200 sectors, d 3..8, "
                        "n 65521, 16 shifts, orders eps^-2..eps^0, deformed contour, FP64 complex",
            "value": evals * steps / el, "unit": "complex evals/s",
            "ms_per_step": el / steps * 1e3, "kernel_ms": kernel_ms / max(launches, 1),
            "evals_per_step": evals, "lambda_choice_s": choose_s,
            "sectors_lambda_halved_presample": int(np.count_nonzero(halv)),
            "sectors_lambda_halved_full_n": int(np.count_nonzero(halv2)),
            "sectors_unfixed": int(rc2 != 0),
            "sectors_violating_at_full_n": int(np.count_nonzero(viol)),
            "scan_wall": workflow,
            "fp32_bulk": {"value": evals * steps / el32, "unit": "complex evals/s",
                          "ms_per_step": el32 / steps * 1e3, "kernel_ms": k32 / max(l32, 1),
                          "speedup_vs_fp64": el / el32,
                          "rel_dev_vs_fp64": {"median": float(np.median(rel)),
                                              "p99": float(np.quantile(rel, 0.99)),
                                              "max": float(rel.max())},
                          "dev_over_stated_error_max": float(np.max(
                              dev / np.maximum(np.hypot(e32[..., 0], e32[..., 1]), 1e-300))),
                          "dev_over_fp64_shift_error_max": float(np.max(dev / np.maximum(err, 1e-300))),
                          "sectors_violating_at_full_n": int(np.count_nonzero(viol32))}}


def scan_flow_leg(qmc, torch, n_points: int = 10, train_points: int = 3, batches: int = 16,
                  epochs: int = 3):
    """Kinematics-conditioned flows on the physical scan: one conditional flow per base
    sector, its networks fed the scaled invariants ((s1, s2) - 5.5) / 4.5, trained on the
    deformed integrand's samples (one shift, n = 65521) of the first train_points
    kinematic points, then applied at every point of the scan; per (sector, point) the
    flow is kept only where its shift variance at equal n is lower than plain QMC's
    (the fallback).  Reports training time, the share of instances that keep the flow,
    variance ratios, the cost of the flow-transformed evaluation and sign-check counts."""
    import numpy as np
    import workloads
    train_points = max(1, min(train_points, n_points - 1))   # leave unseen points
    prob = workloads.physical_scan(seed=0, n_points=n_points)
    kin = prob.kinematics
    nb = len(prob.sectors) // n_points
    plan = qmc.Plan(prob)
    plan.choose_deformation(4099)
    plan.choose_deformation(65521)
    _, m0, e0 = plan.integrate(check=False)
    plan.enable_timing(True)
    plan.integrate(check=False)
    k_plain, _ = plan.read_timing()
    plan.enable_timing(False)
    cond = (kin - 5.5) / 4.5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flows, jobs = [], []
    for b in range(nb):
        sec = prob.sectors[b]
        xs, ws, cs = [], [], []
        for pnt in range(train_points):
            x, w = plan.flow_samples(pnt * nb + b, sec.n, sec.a, shift=0)
            xs.append(x)
            ws.append(w)
            cs.append(torch.tensor(cond[pnt], dtype=torch.float64, device="cuda")
                      .reshape(1, 2).expand(sec.n, 2))
        fl = qmc.flow.Flow(sec.d, params=qmc.flow.glorot_params(sec.d, seed=b, n_cond=2), n_cond=2)
        jobs.append((fl, torch.cat(xs), torch.cat(ws),
                     {"batches": batches, "epochs": epochs, "lr": 2e-3,
                      "cond": torch.cat(cs).contiguous()}))
        flows.append(fl)
    train_flows(torch, jobs)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    for s in range(len(prob.sectors)):
        pnt, b = divmod(s, nb)
        plan.attach_flow(s, flows[b], cond=cond[pnt])
    _, m1, e1 = plan.integrate(check=False)
    viol = plan.sign_violations()
    plan.enable_timing(True)
    plan.integrate(check=False)
    k_flow, _ = plan.read_timing()
    plan.enable_timing(False)
    v0 = (e0.cpu().numpy() ** 2).sum(axis=(1, 2))
    v1 = (e1.cpu().numpy() ** 2).sum(axis=(1, 2))
    ratio = v0 / np.maximum(v1, 1e-300)        # > 1: the flow lowers the shift variance
    keep = (ratio > 1.0) & (viol == 0)         # fallback: plain QMC elsewhere
    train_mask = np.zeros(len(prob.sectors), dtype=bool)
    train_mask[: train_points * nb] = True
    cost = k_flow / k_plain
    return {"workload": f"physical_scan: {n_points} kinematic points x {nb} sectors; one "
                        f"conditional flow per base sector (features (s1, s2)), trained on "
                        f"{train_points} points x 65521 samples ({batches} batches x {epochs} "
                        f"epochs, four flows at a time on separate streams), applied at every "
                        f"point",
            "training_wall_s": train_s,
            "instances_flow_kept": int(keep.sum()), "instances": int(len(keep)),
            "kept_at_unseen_points": int(keep[~train_mask].sum()),
            # kept and cheaper to a given error than plain QMC (sqrt of the variance ratio
            # above the cost ratio, the n^-2 variance decay of the allocation)
            "instances_flow_pays": int(np.count_nonzero(keep & (np.sqrt(ratio) > cost))),
            "variance_ratio_plain_over_flow": {"median": float(np.median(ratio)),
                                               "max": float(ratio.max())},
            "cost_ratio_flow_over_plain": float(cost),
            "flow_complex_evals_per_s": prob.evals() / (k_flow / 1e3),
            "sectors_violating_with_flow": int(np.count_nonzero(viol))}


def flow_leg(qmc, torch, batches: int = 64, epochs: int = 3):
    """Learned transform against korobov3 on the d = 6 sectors of the two-loop integral:
    per sector a flow trained on 1e6 QMC samples (one shift, n = nextprime(1e6)), then the
    shift variance at each sector's own n with and without the flow (32 shifts), the
    training wall time, the flow-integrated throughput and its matrix-core rate."""
    import numpy as np
    import workloads
    full = workloads.two_loop_integral(seed=0)
    idx = [s for s, sec in enumerate(full.sectors) if sec.d == 6]
    prob = workloads.Problem(sectors=[full.sectors[s] for s in idx], order_lo=full.order_lo,
                             m=full.m, shifts=[full.shifts[s] for s in idx])
    n_train = workloads.next_prime(1000000)
    plan = qmc.Plan(prob, n_max=max(n_train, max(s.n for s in prob.sectors)))
    _, m0, e0 = plan.integrate()
    plan.enable_timing(True)
    plan.integrate()
    k_plain, _ = plan.read_timing()
    plan.enable_timing(False)
    cands = np.arange(2, 2 + 64, dtype=np.uint64) * 15485863 % np.uint64(n_train)
    a_train, _ = plan.korobov_search(n_train, 6, [int(c) for c in cands if c > 1])
    flows, jobs = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(len(idx)):
        x, w = plan.flow_samples(s, n_train, a_train, shift=0)
        fl = qmc.flow.Flow(6, seed=s)
        jobs.append((fl, x, w, {"batches": batches, "epochs": epochs, "lr": 2e-3}))
        flows.append(fl)
    train_flows(torch, jobs)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    for s, fl in enumerate(flows):
        plan.attach_flow(s, fl)
    _, m1, e1 = plan.integrate()
    plan.enable_timing(True)
    plan.integrate()
    k_flow, _ = plan.read_timing()
    plan.enable_timing(False)
    v0 = (e0.cpu().numpy() ** 2).sum(axis=1)
    v1 = (e1.cpu().numpy() ** 2).sum(axis=1)
    ratio = v0 / v1                      # > 1: the flow lowers the shift variance
    evals = prob.evals()
    cost = k_flow / k_plain
    flops_eval = 4 * 2 * (6 * 64 + 64 * 64 + 64 * 12)
    return {"workload": f"{len(idx)} d=6 sectors of two_loop_integral, flows trained on "
                        f"{n_train} samples each ({batches} batches x {epochs} epochs, four "
                        f"flows at a time on separate streams)",
            "variance_ratio_plain_over_flow": {"median": float(np.median(ratio)),
                                               "min": float(ratio.min()),
                                               "max": float(ratio.max())},
            "sectors_flow_wins": int(np.count_nonzero(ratio > 1.0)),
            "cost_ratio_flow_over_plain": float(cost),
            # work to a given error under the n^-2 variance decay the allocation assumes:
            # (cost per evaluation) x (lattice size), the size scaling as sqrt(variance)
            "cost_adjusted_ratio_median": float(np.median(np.sqrt(ratio) / cost)),
            "training_wall_s": train_s,
            "flow_evals_per_s": evals / (k_flow / 1e3), "plain_evals_per_s": evals / (k_plain / 1e3),
            "flow_network_tflops": evals * flops_eval / (k_flow / 1e3) / 1e12,
            "flow_network_frac_of_bf16_peak": evals * flops_eval / (k_flow / 1e3) / 2.5e15}


def one_loop_leg(qmc, torch, steps: int = 3):
    """Throughput variant of the one-loop sector: the same integrand (x1^(1/2) U^-1
    F^(-1-eps), two orders, korobov3, 16 shifts) on a lattice of n = 2^31 - 1 points whose
    Korobov parameter minimises P_2 over 64 random candidates (device search, timed
    separately), in FP64: first on the table-driven kernel (the general integrand path:
    the x1^(1/2) factor), then on the plan-specialised one at the autotuner's launch shape
    (compilation and the search, on a lattice of 2^26 points, outside the timing)."""
    import numpy as np
    import workloads
    n = 2 ** 31 - 1
    prob = workloads.one_loop_sector(seed=0, n=n)
    plan = qmc.Plan(prob, n_max=n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a, p2 = plan.korobov_search(n, 3, [int(c) for c in prob.sectors[0].a_candidates])
    search_s = time.perf_counter() - t0

    def measure():
        plan.integrate(n=[n], a=[a])                   # warm-up
        times, kms = [], []
        for _ in range(steps):
            plan.enable_timing(True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, mean, err = plan.integrate(n=[n], a=[a], check=False)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
            kms.append(plan.read_timing()[0])
            plan.enable_timing(False)
        plan.check_status()
        return (float(np.median(times)), float(np.median(kms)),
                mean.cpu().numpy()[0], err.cpu().numpy()[0])

    evals = n * prob.m
    t_tab, k_tab, m_tab, e_tab = measure()
    spec_s = plan.specialize()
    n_tune = workloads.next_prime(1 << 26)
    tune = plan.autotune(n=[n_tune], a=[12345], reps=3, use_cache=False)
    t_gen, k_gen, mean, err = measure()
    return {"workload": "one_loop_sector: d = 3, n = 2^31 - 1, a = argmin P_2 over 64 random "
                        "candidates, 16 shifts, 2 orders, korobov3, FP64",
            "a": a, "p2": p2, "p2_search_s": search_s,
            "value": evals / t_gen, "unit": "evals/s", "ms_per_step": t_gen * 1e3,
            "kernel_ms": k_gen, "evals_per_step": evals,
            "kernel": "plan-specialised", "specialize_seconds": spec_s,
            "launch": {k: tune[k] for k in ("block", "shift_tile", "shifts_per_pass",
                                            "target_blocks")},
            "table_driven": {"value": evals / t_tab, "ms_per_step": t_tab * 1e3,
                             "kernel_ms": k_tab,
                             "max_rel_diff_of_estimates": float(np.max(np.abs(m_tab - mean) /
                                                                       np.abs(mean)))},
            "estimate": [float(v) for v in mean], "error": [float(v) for v in err]}


def two_loop_problem(qmc, torch):
    """The two-loop workload with every sector's Korobov parameter chosen on the device:
    the P_2 minimiser over the sector's 64 seeded candidates (ties: smallest a).
    Returns (problem, seconds of the search)."""
    import workloads
    prob = workloads.two_loop_integral(seed=0)
    plan = qmc.Plan(prob)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sec in prob.sectors:
        sec.a = plan.korobov_search(sec.n, sec.d, [int(c) for c in sec.a_candidates])[0]
    dt = time.perf_counter() - t0
    del plan
    return prob, dt


def median_leg(qmc, torch, r: int = 11, seed: int = 0):
    """Median QMC rule (Sec. 2.2): per sector r generating vectors drawn from U_n and the
    median of their unshifted estimates, all candidates of all sectors in one launch,
    against the P_2-searched Korobov vectors (the benchmark's lattices: argmin of P_2 over
    each sector's 64 candidates) on the two-loop integral, both at each sector's own n
    with the same 32 shifts.  Reports the selection time, its cost in units of one
    32-shift integration, the selection throughput and the per-sector ratio of shift
    errors (all epsilon orders, summed in quadrature)."""
    import numpy as np
    import workloads
    prob, _ = two_loop_problem(qmc, torch)
    plan = qmc.Plan(prob)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 29])))
    cands = np.zeros((plan.S, r, qmc.QMC_MAX_DIM), dtype=np.uint64)
    for s, sec in enumerate(prob.sectors):
        cands[s, :, :sec.d] = workloads.median_candidates(rng, sec.n, sec.d, r)
    _, _, e0 = plan.integrate()
    plan.median_lattice(r=r, candidates=cands)             # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.integrate()
    torch.cuda.synchronize()
    t_int = time.perf_counter() - t0
    t0 = time.perf_counter()
    z, _, _ = plan.median_lattice(r=r, candidates=cands)   # synchronous
    t_sel = time.perf_counter() - t0
    _, _, e1 = plan.integrate(z=z)
    v0 = np.sqrt((e0.cpu().numpy() ** 2).sum(axis=1))
    v1 = np.sqrt((e1.cpu().numpy() ** 2).sum(axis=1))
    ratio = v1 / v0                       # < 1: the median rule's lattice is better
    points = sum(sec.n for sec in prob.sectors)
    return {"workload": f"two_loop_integral ({plan.S} sectors), r = {r} candidates per sector "
                        f"from U_n, each sector's own n, 32 shifts after selection; baseline: "
                        f"Korobov vectors with a = argmin P_2 over 64 candidates",
            "selection_wall_s": t_sel, "integration_wall_s": t_int,
            "selection_cost_in_integrations": t_sel / t_int,
            "selection_evals_per_s": r * points / t_sel,
            "error_ratio_median_over_korobov": {"median": float(np.median(ratio)),
                                                "min": float(ratio.min()),
                                                "max": float(ratio.max())},
            "sectors_median_rule_better": int(np.count_nonzero(ratio < 1.0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--block", type=int, default=0, help="workgroup size (0 = library default)")
    ap.add_argument("--tile", type=int, default=0, help="shifts per workgroup (0 = default)")
    ap.add_argument("--spp", type=int, default=0, help="shifts per pass (0 = default)")
    ap.add_argument("--target", type=int, default=0,
                    help="workgroups a launch aims at (0 = default); with --block/--tile/--spp "
                         "it fixes the launch shape and skips the autotuner")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-integrand measurement")
    ap.add_argument("--no-specialize", action="store_true",
                    help="time the table-driven kernels only (no plan-specialised kernels)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shape (no autotuner search)")
    ap.add_argument("--no-amp", action="store_true", help="skip the amplitude wall-time leg")
    ap.add_argument("--no-flow", action="store_true", help="skip the learned-transform leg")
    ap.add_argument("--no-median", action="store_true", help="skip the median-rule leg")
    ap.add_argument("--no-one-loop", action="store_true",
                    help="skip the one-loop throughput leg (n = 2^31 - 1)")
    ap.add_argument("--no-scan-flow", action="store_true",
                    help="skip the kinematics-conditioned flow leg on the physical scan")
    ap.add_argument("--scan-points", type=int, default=10,
                    help="kinematic points of the deformed-contour scan leg (0 = skip)")
    ap.add_argument("--amp-repeats", type=int, default=3)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the lattice QMC "
                                   "path has no multi-GPU mode (--gpus must be 1)"}))
        sys.exit(2)

    import torch
    import workloads
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2305_19768_amd as qmc

    torch.cuda.set_device(0)
    prob, p2_search_s = two_loop_problem(qmc, torch)
    t0 = time.perf_counter()
    plan = qmc.Plan(prob, block=args.block, shift_tile=args.tile, shifts_per_pass=args.spp)
    explicit = bool(args.block or args.tile or args.spp or args.target)
    if explicit:
        plan.set_launch_shape(args.block or 256, args.tile or 16, args.spp or 2,
                              args.target or 16384)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    spec_s = None
    if not args.no_specialize:
        spec_s = plan.specialize()          # generated per-sector kernels, before any timing
        print(f"# specialised kernels compiled in {spec_s:.1f} s", file=sys.stderr, flush=True)
    tune = None
    if not (args.no_tune or explicit):
        t0 = time.perf_counter()
        tune = plan.autotune(reps=4)        # launch-shape search, outside the timed region
        tune["seconds"] = time.perf_counter() - t0
        print(f"# autotuned launch shape {tune}", file=sys.stderr, flush=True)
    S, m, K = plan.S, plan.m, plan.K
    out = (torch.empty((S, m, K), dtype=torch.float64, device="cuda"),
           torch.empty((S, K), dtype=torch.float64, device="cuda"),
           torch.empty((S, K), dtype=torch.float64, device="cuda"))
    for _ in range(args.warmup):
        plan.integrate(out=out, check=False)
    torch.cuda.synchronize()
    plan.check_status()
    print(f"# warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    plan.enable_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.integrate(out=out, check=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms, launches = plan.read_timing()
    plan.enable_timing(False)
    plan.check_status()
    mean64, err64 = out[1].cpu().numpy().copy(), out[2].cpu().numpy().copy()

    table = None
    if spec_s is not None:
        # the same plan and launch shape on the table-driven kernels, for comparison
        plan.specialize(off=True)
        for _ in range(args.warmup):
            plan.integrate(out=out, check=False)
        plan.enable_timing(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            plan.integrate(out=out, check=False)
        torch.cuda.synchronize()
        et = time.perf_counter() - t1
        kt_ms, kt_n = plan.read_timing()
        plan.enable_timing(False)
        plan.check_status()
        table = {"value": prob.evals() * args.steps / et, "unit": "evals/s",
                 "ms_per_step": et / args.steps * 1e3, "kernel_ms": kt_ms / max(kt_n, 1),
                 "note": "table-driven kernels (dense degree-3 Horner), same plan and shape"}

    fp32 = None
    if not args.no_fp32:
        plan32 = qmc.Plan(prob, precision=qmc.QMC_PREC_FP32, block=args.block,
                          shift_tile=args.tile, shifts_per_pass=args.spp)
        if spec_s is not None:
            plan32.specialize()
        tune32 = None
        if explicit:
            plan32.set_launch_shape(args.block or 256, args.tile or 16, min(args.spp or 2, 2),
                                    args.target or 16384)
        elif tune is not None:
            tune32 = plan32.autotune(reps=4)
        for _ in range(args.warmup):
            plan32.integrate(out=out, check=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            plan32.integrate(out=out, check=False)
        torch.cuda.synchronize()
        e32 = time.perf_counter() - t1
        plan32.check_status()
        import numpy as np
        mean32 = out[1].cpu().numpy()
        err32 = out[2].cpu().numpy()   # stated error: shift error + the FP32 rounding bound
        dev = np.abs(mean32 - mean64)
        rel = dev / np.abs(mean64)
        flops32 = sum(algorithmic_flops(sec, m) * sec.n * m for sec in prob.sectors)
        fp32 = {"value": prob.evals() * args.steps / e32, "unit": "evals/s",
                "ms_per_step": e32 / args.steps * 1e3,
                "roofline": {"bound": "alu", "achieved": flops32 / (e32 / args.steps) / 1e12,
                             "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": flops32 / (e32 / args.steps) / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                             "timing": "wall clock of the step"},
                "note": "FP32 integrand, FP64 lattice points and accumulation",
                "launch": tune32, "specialised": spec_s is not None,
                # the FP32 form's error against the FP64 form, per result (sector, order)
                "rel_dev_vs_fp64": {"median": float(np.median(rel)), "max": float(rel.max()),
                                    "per_sector_max": [float(f"{v:.3g}") for v in rel.max(axis=1)]},
                # the deviation against the error the FP32 form states for itself (must be
                # <= 1), and against the FP64 form's shift error alone (context)
                "dev_over_stated_error": {"max": float((dev / err32).max()),
                                          "median": float(np.median(dev / err32))},
                "dev_over_fp64_shift_error_max": float((dev / err64).max())}
        del plan32

    if args.copy_probe:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    evals = prob.evals()
    value = evals * args.steps / elapsed
    flops_launch = sum(algorithmic_flops(sec, m) * sec.n * m for sec in prob.sectors)
    k_s = kernel_ms / max(launches, 1) / 1e3
    achieved = flops_launch / k_s / 1e12
    traffic = measured_traffic()
    result = {
        "metric": "integrand evals/s (FP64 vs FP32) and wall time to 1e-4 rel. amplitude error",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded two-loop-like sectors; the paper's integrands are not "
                "available)",
        "config": {"workload": "two_loop_integral: 40 sectors, d 4..6, n 1e5..1e7 prime, "
                               "Korobov a = argmin P_2 over 64 candidates, 32 shifts, orders "
                               "eps^-2..eps^0, korobov3, FP64",
                   "sectors": S, "shifts": m, "orders": K, "evals_per_step": evals,
                   "lattice_points_per_step": int(sum(s.n for s in prob.sectors))},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic,
                     "kernel": (("qmc_gen_d{4,5,6}_f64_s%d (plan-specialised" % plan.launch_shape()["shifts_per_pass"])
                                if spec_s is not None
                                else "qmc_integrate_kernel<D,3,S> (table-driven") +
                               "; d = 4, 5, 6 concurrent launches, kernel_ms is their joint span)",
                     "kernel_ms": kernel_ms / max(launches, 1),
                     "algorithmic_flops_per_launch": flops_launch,
                     "flops_per_eval": flops_launch / evals},
        "fp32": fp32,
        "table_driven": table,
        "plan_seconds": plan_s,
        "specialize_seconds": spec_s,
        "korobov_p2_search_seconds": p2_search_s,
        "launch": plan.launch_shape(),
        "autotune": tune,
        "paper_figures": PAPER_FIGURES,
    }
    if not args.no_one_loop:
        result["one_loop_throughput"] = one_loop_leg(qmc, torch)
    if not args.no_amp:
        result["amplitude_time_to_1e-4"] = amplitude_leg(qmc, torch, args.amp_repeats)
    if not args.no_flow:
        result["learned_transform"] = flow_leg(qmc, torch)
    if not args.no_median:
        result["median_rule"] = median_leg(qmc, torch)
    if args.scan_points > 0:
        result["physical_scan"] = scan_leg(qmc, torch, args.scan_points, max(1, args.steps // 4))
        if not args.no_scan_flow:
            result["physical_scan"]["conditional_flow"] = scan_flow_leg(qmc, torch, args.scan_points)
    if not args.no_cpu:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        result["cpu_baseline"] = cpu_baseline(prob, threads)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
