"""Pins of the coupling-flow oracle (CPU only): identity at initialisation, exact
invertibility, the log-determinant against finite differences, unbiasedness of the
transformed integral (Gauss-Legendre), the training gradient against finite differences,
the first Adam step in closed form, bfloat16 rounding, and that training on a peaked
integrand lowers the variance of the transformed integrand."""
import numpy as np
import pytest

from oracle import flow as F


def _params(d, seed=1, scale=1.5):
    return F.init_params(d, seed=seed, zero_last=False, scale=scale)


def test_bf16_rounding():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -2.5, 1 + 2 ** -7, 3.0e38])
    r = F.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0                 # tie to even
    assert r[2] == 1 + 2 ** -7 and r[3] == -2.5 and r[4] == 1 + 2 ** -7
    assert np.isfinite(r[5])
    x = np.random.default_rng(0).normal(size=1000)
    assert np.all(np.abs(F.bf16(x) - x) <= 2 ** -8 * np.abs(x))   # unit roundoff, 8 bits


def test_identity_at_initialisation():
    d = 6
    p = F.init_params(d, seed=0)
    u = np.random.default_rng(1).uniform(0.01, 0.99, size=(50, d))
    x, logJ = F.sampling_direction(p, u)
    assert np.allclose(x, u, rtol=0, atol=1e-15) and np.allclose(logJ, 0, atol=1e-12)


@pytest.mark.parametrize("d", [2, 5, 6])
def test_invertibility_and_logdet_cancel(d):
    p = _params(d)
    u = np.random.default_rng(2).uniform(0.02, 0.98, size=(40, d))
    x, logJ = F.sampling_direction(p, u)
    assert np.max(np.abs(x - u)) > 1e-3                # a non-trivial map
    u2, logq = F.density_direction(p, x)
    assert np.allclose(u2, u, rtol=0, atol=1e-12)
    assert np.allclose(logJ + logq, 0, atol=1e-10)


def test_logdet_against_finite_differences():
    d = 4
    p = _params(d, seed=3)
    rng = np.random.default_rng(3)
    for u in rng.uniform(0.1, 0.9, size=(5, d)):
        _, logJ = F.sampling_direction(p, u[None, :])
        h = 1e-6
        Jm = np.empty((d, d))
        for k in range(d):
            e = np.zeros(d)
            e[k] = h
            xp, _ = F.sampling_direction(p, (u + e)[None, :])
            xm, _ = F.sampling_direction(p, (u - e)[None, :])
            Jm[:, k] = (xp[0] - xm[0]) / (2 * h)
        assert abs(np.log(abs(np.linalg.det(Jm))) - logJ[0]) < 1e-6


def test_transformed_integral_is_unbiased():
    # int f(T(u)) J_T(u) du = int f(x) dx for f = x1^2 x2 (exact 1/6), and the model
    # density integrates to one, by 2-D Gauss-Legendre; the transformed integrand has
    # power-law behaviour at the faces (logit-space scaling), so the rule converges
    # algebraically: the errors must shrink steadily towards zero
    p = _params(2, seed=4, scale=2.0)
    errs = []
    for N in (400, 800):
        g, w = np.polynomial.legendre.leggauss(N)
        g = 0.5 * (g + 1)
        w = 0.5 * w
        U = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2)
        Wt = np.outer(w, w).reshape(-1)
        x, logJ = F.sampling_direction(p, U)
        val = np.sum(Wt * x[:, 0] ** 2 * x[:, 1] * np.exp(logJ))
        mass = np.sum(Wt * np.exp(F.density_direction(p, U)[1]))
        errs.append((abs(val - 1 / 6), abs(mass - 1.0)))
    assert errs[1][0] < 1e-7 and errs[1][1] < 2e-6
    assert errs[0][0] > 2.5 * errs[1][0] and errs[0][1] > 2.5 * errs[1][1]


def test_gradient_against_finite_differences():
    d = 3
    p = _params(d, seed=5)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.05, 0.95, size=(64, d))
    w = rng.uniform(0.1, 2.0, size=64)
    L, grads = F.weighted_nll_and_grad(p, x, w)
    _, logq = F.density_direction(p, x)
    assert abs(L + np.sum(w * logq) / np.sum(w)) < 1e-12
    for (layer, which, idx) in [(0, 0, (3, 1)), (1, 2, (10, 20)), (3, 4, (1, 7)), (2, 5, (2,)),
                                (0, 1, (5,))]:
        h = 1e-6
        pp = [[a.copy() for a in q] for q in p]
        pp[layer][which][idx] += h
        lp = -np.sum(w * F.density_direction(pp, x)[1]) / np.sum(w)
        pp[layer][which][idx] -= 2 * h
        lm = -np.sum(w * F.density_direction(pp, x)[1]) / np.sum(w)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grads[layer][which][idx]) < 1e-6 * (1 + abs(fd)), (layer, which, idx)


def test_first_adam_step_closed_form():
    p = _params(2, seed=6)
    g = [[np.full_like(a, 0.5) * np.sign(np.arange(a.size).reshape(a.shape) % 3 - 1)
          for a in q] for q in p]
    p1, st = F.adam_step(p, g, F.adam_init(p), lr=1e-2)
    for q0, q1, gq in zip(p, p1, g):
        for a0, a1, ga in zip(q0, q1, gq):
            # m_hat = g, v_hat = g^2: the step is lr * g / (|g| + eps)
            assert np.allclose(a1 - a0, -1e-2 * ga / (np.abs(ga) + 1e-8), atol=1e-15)
    assert st[0] == 1


def test_training_lowers_variance_of_peaked_integrand():
    d = 2
    rng = np.random.default_rng(7)

    def f(x):
        return np.exp(-40 * ((x[:, 0] - 0.3) ** 2 + (x[:, 1] - 0.6) ** 2))

    p = F.init_params(d, seed=7)
    st = F.adam_init(p)
    xs = rng.uniform(size=(4096, d))
    ws = f(xs)
    for _ in range(150):
        _, g = F.weighted_nll_and_grad(p, xs, ws)
        p, st = F.adam_step(p, g, st, lr=3e-3)
    u = rng.uniform(size=(20000, d))
    x, logJ = F.sampling_direction(p, u)
    gval = f(x) * np.exp(logJ)
    plain = f(u)
    assert abs(gval.mean() - plain.mean()) < 4 * gval.std() / np.sqrt(len(u))
    assert gval.var() < 0.5 * plain.var()


# ------------------------------------------------------ conditional flows (scan)
def test_conditional_flow_reduces_and_depends_on_condition():
    # zero weights on the conditioning columns give the unconditional flow exactly;
    # non-zero ones make the map depend on the condition, and every conditional map is
    # still an exact bijection with cancelling log-determinants
    d, c = 4, 2
    p = F.init_params(d, seed=8, zero_last=False, scale=1.5, n_cond=c)
    p0 = [[a.copy() for a in q] for q in p]
    for q in p0:
        q[0][:, d:] = 0.0
    pu = [[q[0][:, :d]] + q[1:] for q in p0]
    u = np.random.default_rng(8).uniform(0.02, 0.98, size=(30, d))
    cond = np.array([0.3, -0.7])
    x0, l0 = F.sampling_direction(p0, u, cond=cond)
    xu, lu = F.sampling_direction(pu, u)
    assert np.array_equal(x0, xu) and np.array_equal(l0, lu)
    x1, l1 = F.sampling_direction(p, u, cond=cond)
    x2, _ = F.sampling_direction(p, u, cond=np.array([-0.5, 0.9]))
    assert np.max(np.abs(x1 - x2)) > 1e-3
    u1, q1 = F.density_direction(p, x1, cond=cond)
    assert np.allclose(u1, u, atol=1e-12) and np.allclose(l1 + q1, 0, atol=1e-10)
    # per-point conditions: row t of the batch uses cond[t]
    cs = np.random.default_rng(9).uniform(-1, 1, size=(30, c))
    xb, _ = F.sampling_direction(p, u, cond=cs)
    for t in (0, 7, 29):
        xt, _ = F.sampling_direction(p, u[t:t + 1], cond=cs[t])
        assert np.allclose(xb[t], xt[0], atol=1e-15)


def test_conditional_gradient_against_finite_differences():
    d, c = 3, 2
    p = F.init_params(d, seed=10, zero_last=False, scale=1.0, n_cond=c)
    rng = np.random.default_rng(10)
    x = rng.uniform(0.05, 0.95, size=(64, d))
    w = rng.uniform(0.1, 2.0, size=64)
    cs = rng.uniform(-1, 1, size=(64, c))
    L, grads = F.weighted_nll_and_grad(p, x, w, cond=cs)
    for (layer, idx) in [(0, (3, d)), (2, (10, d + 1)), (1, (5, 0))]:
        h = 1e-6
        pp = [[a.copy() for a in q] for q in p]
        pp[layer][0][idx] += h
        lp = -np.sum(w * F.density_direction(pp, x, cond=cs)[1]) / np.sum(w)
        pp[layer][0][idx] -= 2 * h
        lm = -np.sum(w * F.density_direction(pp, x, cond=cs)[1]) / np.sum(w)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grads[layer][0][idx]) < 1e-6 * (1 + abs(fd)), (layer, idx)
    v = F.flatten(p)
    assert len(v) == 4 * (64 * (d + c) + 64 + 64 * 64 + 64 + 2 * d * 64 + 2 * d)
    back = F.unflatten(v.astype(np.float64), d, n_cond=c)
    assert all(np.array_equal(a.astype(np.float32), b.astype(np.float32))
               for q, r in zip(p, back) for a, b in zip(q, r))


def test_deformed_sums_through_identity_flow_equal_the_contour_sums():
    # the flow composition on the deformed contour: with an identity flow the sums are
    # those of the plain deformed-contour oracle (a different code path in C)
    import oracle
    import workloads as W
    prob = W.physical_scan(seed=2, n_points=1, n_sectors=2, d_lo=3, d_hi=4, n=1009, m=4)
    for s, sec in enumerate(prob.sectors):
        sec.deform_lambda, _ = oracle.choose_lambda(sec, prob.shifts[s], 0.5, 1009, sec.a)
        p = F.init_params(sec.d, seed=s, n_cond=2)          # identity (zero last layer)
        Q, S = F.sector_sums(sec, prob.shifts[s], p, bf=True, cond=np.array([0.1, 0.2]),
                             deformed=True)
        Qd, Sd, _, _ = oracle.sector_sums_deformed(sec, prob.shifts[s])
        assert np.allclose(Q, Qd, rtol=1e-12, atol=1e-12 * np.max(Sd))
