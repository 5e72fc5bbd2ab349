"""GPU parity of the learned coupling-flow transform with the oracle (oracle/flow.py).

The device network runs in bfloat16 with float32 accumulation; the oracle in its
bfloat16 mode rounds the same values but sums exactly, so outputs agree to the float32
accumulation order (tolerances below), except where a hidden activation lands on the
other side of a bfloat16 rounding boundary.  Gradients are compared with the float64
oracle gradient (bfloat16 operands in the device products), Adam exactly in float32
arithmetic, training samples and flow-integrated sums element by element.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import flow as OF

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qmc():
    import __graft_entry__ as g
    g._ensure_built()
    import torch
    import paper_2305_19768_amd as q
    torch.cuda.set_device(0)
    return q


def _random_flow(qmc, d, seed, scale=1.5):
    p = OF.init_params(d, seed=seed, zero_last=False, scale=scale)
    v = OF.flatten(p)
    fl = qmc.flow.Flow(d, params=v)
    return fl, OF.unflatten(v.astype(np.float64), d)


@pytest.mark.parametrize("d", [1, 2, 5, 6, 8])
def test_transform_both_directions_match_oracle(qmc, d):
    fl, p = _random_flow(qmc, d, seed=d)
    u = np.random.default_rng(d).uniform(0.01, 0.99, size=(1000, d))
    x, logJ = fl.transform(u, qmc.flow.SAMPLE)
    x, logJ = x.cpu().numpy(), logJ.cpu().numpy()
    ox, olJ = OF.sampling_direction(p, u, bf=True)
    # agreement to float32 accumulation, except points where a hidden activation rounds
    # to the neighbouring bfloat16 value on one side: a small fraction, bounded effect
    dx = np.abs(x - ox)
    far = np.mean(np.any(dx > 1e-6, axis=1))
    print("d", d, "median |dx|", np.median(dx), "max", dx.max(), "points off", far, flush=True)
    assert np.median(dx) < 1e-7 and far < 0.03 and dx.max() < 5e-2
    dl = np.abs(logJ - olJ)
    assert np.median(dl) < 1e-6 and np.mean(dl > 1e-5) < 0.03
    # density direction on the device inverts the sampling direction up to that noise
    u2, logq = fl.transform(x, qmc.flow.DENSITY)
    u2, logq = u2.cpu().numpy(), logq.cpu().numpy()
    ou2, olq = OF.density_direction(p, x, bf=True)
    du = np.abs(u2 - ou2)
    assert np.median(du) < 1e-7 and np.mean(np.any(du > 1e-6, axis=1)) < 0.03
    assert np.median(np.abs(logq + logJ)) < 1e-4


def test_identity_flow_is_exact(qmc):
    d = 6
    fl = qmc.flow.Flow(d, params=qmc.flow.glorot_params(d, seed=1, zero_last=True))
    u = np.random.default_rng(0).uniform(0.001, 0.999, size=(300, d))
    x, logJ = fl.transform(u)
    assert np.max(np.abs(x.cpu().numpy() - u)) < 1e-14
    assert np.max(np.abs(logJ.cpu().numpy())) < 1e-12


@pytest.mark.parametrize("count", [2048, 777])
def test_gradient_and_adam_match_oracle(qmc, count):
    d = 3
    fl, p = _random_flow(qmc, d, seed=5, scale=1.0)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.05, 0.95, size=(count, d))
    w = rng.uniform(0.1, 2.0, size=count)
    loss = fl.gradient(x, w)
    L, g = OF.weighted_nll_and_grad(p, x, w)
    _, olq = OF.density_direction(p, x, bf=True)
    Lb = -np.sum(w * olq) / np.sum(w)
    assert abs(loss - Lb) <= 1e-4 * (1 + abs(Lb)), (loss, Lb, L)
    prm, grd = fl.read()
    og = OF.flatten(g).astype(np.float64)
    cos = float(np.dot(grd, og) / (np.linalg.norm(grd) * np.linalg.norm(og)))
    rel = float(np.linalg.norm(grd - og) / np.linalg.norm(og))
    print("count", count, "cos", cos, "rel", rel, flush=True)
    assert cos > 0.999 and rel < 5e-2
    # every parameter block receives its gradient (no block left unwritten)
    blocks = OF.unflatten(grd.astype(np.float64), d)
    for layer in blocks:
        for b in (layer[0], layer[2], layer[4], layer[1], layer[3], layer[5]):
            assert np.all(np.isfinite(b)) and np.any(b != 0)
    # one Adam step on the device gradient, against the oracle's update of the same
    fl.adam_step(step=1, lr=1e-2)
    prm1, _ = fl.read()
    ref, _ = OF.adam_step(OF.unflatten(prm.astype(np.float64), d),
                          OF.unflatten(grd.astype(np.float64), d),
                          OF.adam_init(OF.unflatten(prm.astype(np.float64), d)), lr=1e-2)
    assert np.allclose(prm1, OF.flatten(ref), rtol=1e-6, atol=1e-7)


def test_training_samples_match_oracle(qmc):
    rng = np.random.default_rng(8)
    sec = W._two_loop_sector(rng, 4, 4099, 0)
    prob = W.Problem(sectors=[sec], order_lo=-2, m=4, shifts=[W.uniform_shifts(rng, 4, 4)])
    plan = qmc.Plan(prob)
    x, w = plan.flow_samples(0, 4099, sec.a, shift=1)
    x, w = x.cpu().numpy(), w.cpu().numpy()
    z = oracle.korobov_vector(4099, sec.a, 4)
    y = oracle.points(4099, z, prob.shifts[0][1])
    ox, ow = oracle.transform(sec.transform, y)
    Wt = np.prod(ow, axis=1)
    f = oracle.integrand(sec, ox)
    wref = np.where(Wt != 0, Wt * np.sqrt(np.sum(f * f, axis=1)), 0.0)
    assert np.max(np.abs(x - ox)) < 1e-14
    assert np.all(np.abs(w - wref) <= 1e-12 * np.abs(wref) + 1e-300)


def test_flow_integration_matches_oracle(qmc):
    rng = np.random.default_rng(9)
    secs = [W._two_loop_sector(rng, d, W.next_prime(1800 + 300 * d), 0) for d in (3, 5)]
    prob = W.Problem(sectors=secs, order_lo=-2, m=8,
                     shifts=[W.uniform_shifts(rng, 8, s.d) for s in secs])
    plan = qmc.Plan(prob)
    flows = []
    for s, sec in enumerate(secs):
        fl, p = _random_flow(qmc, sec.d, seed=20 + s, scale=0.7)
        plan.attach_flow(s, fl)
        flows.append((fl, p))
    q, _, _ = plan.integrate()
    q = q.cpu().numpy()
    for s, sec in enumerate(secs):
        Q, S = OF.sector_sums(sec, prob.shifts[s], flows[s][1], bf=True)
        dev = np.abs(q[s] - Q) / np.maximum(np.abs(Q), S)
        print("sector", s, "max rel", dev.max(), flush=True)
        assert np.all(dev < 1e-5)
    # detaching restores the plain periodizing transform
    plan.attach_flow(0, None)
    q0, _, _ = plan.integrate()
    Q0, _ = oracle.sector_sums(secs[0], prob.shifts[0])
    assert np.allclose(q0.cpu().numpy()[0], Q0, rtol=1e-12, atol=1e-14)


def test_training_on_gpu_lowers_variance_of_peaked_integrand(qmc):
    # F = 0.02 + sum_j (x_j - 1/2)^2 (monomials), integrand F^-2: a peak at the centre
    d = 2
    f_terms = [(0.02 + 0.25 * d, (0, 0)), (-1.0, (1, 0)), (1.0, (2, 0)), (-1.0, (0, 1)),
               (1.0, (0, 2))]
    sec = W.custom_sector(d, [(1.0, (0, 0))], f_terms, f_pow2=-4, transform="none",
                          n=W.next_prime(200000))
    sec.a = oracle.korobov_search(sec.n, d, np.arange(2, 500, dtype=np.uint64))[0]
    rng = np.random.default_rng(10)
    prob = W.Problem(sectors=[sec], order_lo=0, m=16, shifts=[W.uniform_shifts(rng, 16, d)])
    plan = qmc.Plan(prob)
    _, m0, e0 = plan.integrate()
    x, w = plan.flow_samples(0, sec.n, sec.a, shift=0)
    fl = qmc.flow.Flow(d, params=qmc.flow.glorot_params(d, seed=3))
    hist = fl.train(x, w, batches=16, epochs=6, lr=3e-3)
    print("loss", hist[0], hist[-1], flush=True)
    assert np.all(np.isfinite(hist)) and hist[-1] < hist[0] - 0.1
    # what training optimises: the variance of f(T(u)) J_T(u) under uniform u (the
    # integrand itself evaluated by the oracle at the device-transformed points)
    u = rng.uniform(size=(40000, d))
    xt, logJ = fl.transform(u)
    g = oracle.integrand(sec, xt.cpu().numpy())[:, 0] * np.exp(logJ.cpu().numpy())
    f0 = oracle.integrand(sec, u)[:, 0]
    print("variance plain", f0.var(), "flow", g.var(), flush=True)
    assert g.var() < 0.5 * f0.var()
    assert abs(g.mean() - f0.mean()) < 5 * (g.std() + f0.std()) / np.sqrt(len(u))
    # the lattice rule through the trained flow estimates the same integral
    plan.attach_flow(0, fl)
    _, m1, e1 = plan.integrate()
    m0, e0, m1, e1 = (t.cpu().numpy()[0, 0] for t in (m0, e0, m1, e1))
    print("lattice plain", m0, e0, "flow", m1, e1, flush=True)
    assert abs(m1 - m0) <= 5 * (e0 + e1)


# ------------------------------------------ conditional flows, deformed contour
def _cond_flow(qmc, d, c, seed, scale=1.5):
    p = OF.init_params(d, seed=seed, zero_last=False, scale=scale, n_cond=c)
    v = OF.flatten(p)
    fl = qmc.flow.Flow(d, params=v, n_cond=c)
    return fl, OF.unflatten(v.astype(np.float64), d, n_cond=c)


@pytest.mark.parametrize("d,c", [(5, 2), (3, 4), (8, 2)])
def test_conditional_transform_matches_oracle(qmc, d, c):
    fl, p = _cond_flow(qmc, d, c, seed=30 + d)
    rng = np.random.default_rng(d + 10 * c)
    u = rng.uniform(0.01, 0.99, size=(1000, d))
    cond = rng.uniform(-1.0, 1.0, size=(1000, c))
    x, logJ = fl.transform(u, qmc.flow.SAMPLE, cond=cond)
    x, logJ = x.cpu().numpy(), logJ.cpu().numpy()
    ox, olJ = OF.sampling_direction(p, u, bf=True, cond=cond)
    dx = np.abs(x - ox)
    far = np.mean(np.any(dx > 1e-6, axis=1))
    print("d", d, "c", c, "median |dx|", np.median(dx), "points off", far, flush=True)
    assert np.median(dx) < 1e-7 and far < 0.03 and dx.max() < 5e-2
    dl = np.abs(logJ - olJ)
    assert np.median(dl) < 1e-6 and np.mean(dl > 1e-5) < 0.03
    u2, logq = fl.transform(x, qmc.flow.DENSITY, cond=cond)
    assert np.median(np.abs(u2.cpu().numpy() - u)) < 1e-6
    assert np.median(np.abs(logq.cpu().numpy() + logJ)) < 1e-4
    # the condition matters: other features give another map
    x3, _ = fl.transform(u, qmc.flow.SAMPLE, cond=-cond)
    assert np.median(np.abs(x3.cpu().numpy() - x)) > 1e-4


def test_conditional_gradient_matches_oracle(qmc):
    d, c = 3, 2
    fl, p = _cond_flow(qmc, d, c, seed=40, scale=1.0)
    rng = np.random.default_rng(40)
    x = rng.uniform(0.05, 0.95, size=(2048, d))
    w = rng.uniform(0.1, 2.0, size=2048)
    cond = rng.uniform(-1.0, 1.0, size=(2048, c))
    loss = fl.gradient(x, w, cond=cond)
    L, g = OF.weighted_nll_and_grad(p, x, w, cond=cond)
    _, olq = OF.density_direction(p, x, bf=True, cond=cond)
    Lb = -np.sum(w * olq) / np.sum(w)
    assert abs(loss - Lb) <= 1e-4 * (1 + abs(Lb)), (loss, Lb, L)
    _, grd = fl.read()
    og = OF.flatten(g).astype(np.float64)
    cos = float(np.dot(grd, og) / (np.linalg.norm(grd) * np.linalg.norm(og)))
    rel = float(np.linalg.norm(grd - og) / np.linalg.norm(og))
    print("cos", cos, "rel", rel, flush=True)
    assert cos > 0.999 and rel < 5e-2
    # the conditioning columns of W1 receive their gradient
    blocks = OF.unflatten(grd.astype(np.float64), d, n_cond=c)
    oblk = OF.unflatten(og, d, n_cond=c)
    for l in range(4):
        a, b = blocks[l][0][:, d:], oblk[l][0][:, d:]
        assert np.linalg.norm(a - b) <= 0.1 * np.linalg.norm(b)


def _scan_problem(qmc, n=2003, n_points=2, n_sectors=3, m=8, seed=3):
    prob = W.physical_scan(seed=seed, n_points=n_points, n_sectors=n_sectors, d_lo=3, d_hi=6,
                           n=n, m=m)
    plan = qmc.Plan(prob)
    lam, _, rc = plan.choose_deformation(509)
    assert rc == 0
    for s, sec in enumerate(prob.sectors):
        sec.deform_lambda = float(lam[s])
    return prob, plan


def test_deformed_flow_integration_matches_oracle(qmc):
    prob, plan = _scan_problem(qmc)
    kin = prob.kinematics
    nb = len(prob.sectors) // len(kin)
    flows = {}
    for s, sec in enumerate(prob.sectors):
        pnt, b = divmod(s, nb)
        if b not in flows:
            flows[b] = _cond_flow(qmc, sec.d, 2, seed=50 + b, scale=0.7)
        cond = (kin[pnt] - 5.5) / 4.5
        plan.attach_flow(s, flows[b][0], cond=cond)
    q, _, _ = plan.integrate(check=False)
    q = q.cpu().numpy()
    for s, sec in enumerate(prob.sectors):
        pnt, b = divmod(s, nb)
        Q, S = OF.sector_sums(sec, prob.shifts[s], flows[b][1], bf=True,
                              cond=(kin[pnt] - 5.5) / 4.5, deformed=True)
        g = q[s, :, :, 0] + 1j * q[s, :, :, 1]
        dev = np.abs(g - Q) / np.maximum(np.abs(Q), S)
        print("sector", s, "d", sec.d, "max rel", dev.max(), flush=True)
        assert np.all(dev < 1e-5)
    # detached: back to the plain deformed contour, bit-level parity with the oracle
    for s in range(len(prob.sectors)):
        plan.attach_flow(s, None)
    q0, _, _ = plan.integrate(check=False)
    Q0, S0, _, _ = oracle.sector_sums_deformed(prob.sectors[0], prob.shifts[0])
    g0 = q0.cpu().numpy()[0, :, :, 0] + 1j * q0.cpu().numpy()[0, :, :, 1]
    assert np.all(np.abs(g0 - Q0) <= 1e-12 * np.maximum(np.abs(Q0), S0))


def test_deformed_training_samples_match_oracle(qmc):
    prob, plan = _scan_problem(qmc, n_points=1, n_sectors=2)
    for s, sec in enumerate(prob.sectors):
        x, w = plan.flow_samples(s, 2003, sec.a, shift=1)
        x, w = x.cpu().numpy(), w.cpu().numpy()
        z = oracle.korobov_vector(2003, sec.a, sec.d)
        y = oracle.points(2003, z, prob.shifts[s][1])
        ox, ow = oracle.transform(sec.transform, y)
        Wt = np.prod(ow, axis=1)
        f, _ = oracle.integrand_deformed(sec, ox)
        wref = np.where(Wt != 0, Wt * np.sqrt(np.sum(np.abs(f) ** 2, axis=1)), 0.0)
        assert np.max(np.abs(x - ox)) < 1e-14
        assert np.all(np.abs(w - wref) <= 1e-11 * np.abs(wref) + 1e-300)


def test_conditional_flow_trained_on_scan_lowers_variance(qmc):
    # one conditional flow for a base sector, trained on the deformed integrand's samples
    # of two kinematic points, applied at a third: the flow estimate agrees with plain
    # QMC within the errors, and its shift variance is finite and reported
    prob, plan = _scan_problem(qmc, n=8191, n_points=3, n_sectors=1, m=8, seed=4)
    kin = prob.kinematics
    sec0 = prob.sectors[0]
    xs, ws, cs = [], [], []
    for pnt in (0, 1):
        x, w = plan.flow_samples(pnt, 8191, sec0.a, shift=0)
        xs.append(x)
        ws.append(w)
        cs.append(np.tile((kin[pnt] - 5.5) / 4.5, (8191, 1)))
    import torch
    x = torch.cat(xs)
    w = torch.cat(ws)
    cond = np.concatenate(cs)
    fl = qmc.flow.Flow(sec0.d, params=qmc.flow.glorot_params(sec0.d, seed=5, n_cond=2), n_cond=2)
    hist = fl.train(x, w, batches=8, epochs=4, lr=2e-3, cond=cond)
    assert np.all(np.isfinite(hist))
    _, m0, e0 = plan.integrate(check=False)
    plan.attach_flow(2, fl, cond=(kin[2] - 5.5) / 4.5)
    _, m1, e1 = plan.integrate(check=False)
    m0, e0, m1, e1 = (t.cpu().numpy()[2] for t in (m0, e0, m1, e1))
    v0 = m0[..., 0] + 1j * m0[..., 1]
    v1 = m1[..., 0] + 1j * m1[..., 1]
    err = np.hypot(e0[..., 0], e0[..., 1]) + np.hypot(e1[..., 0], e1[..., 1])
    print("plain", v0, "flow", v1, "err", err, flush=True)
    assert np.all(np.abs(v1 - v0) <= 6 * err)


def test_attach_rejects_a_flow_of_another_shape(qmc):
    prob, plan = _scan_problem(qmc, n_points=1, n_sectors=1)
    d = prob.sectors[0].d
    fl = qmc.flow.Flow(d, n_cond=2)
    fl.n_cond = 0                      # lie about the shape: the header check refuses it
    with pytest.raises(qmc.QmcError, match="attached as"):
        plan.attach_flow(0, fl)
    fl.n_cond = 2
    plan.attach_flow(0, fl, cond=[0.0, 0.5])
    plan.attach_flow(0, None)


def test_training_on_another_stream_matches(qmc):
    """Training launched on a second stream is ordered after the inputs prepared on the
    current stream and before the losses read there: same losses and parameters, bit for
    bit, as on the current stream."""
    import torch
    rng = np.random.default_rng(17)
    x = torch.as_tensor(rng.uniform(0.02, 0.98, size=(4096, 3)), device="cuda")
    w = torch.as_tensor(rng.uniform(0.1, 1.0, size=4096), device="cuda")
    f1 = qmc.flow.Flow(3, seed=5)
    h1 = f1.train(x, w, batches=4, epochs=2, lr=2e-3)
    f2 = qmc.flow.Flow(3, seed=5)
    side = torch.cuda.Stream()          # default priority
    h2 = f2.train(x, w, batches=4, epochs=2, lr=2e-3, stream=side)
    assert np.array_equal(h1, h2)
    assert np.array_equal(f1.read()[0], f2.read()[0])
