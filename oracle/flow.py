"""CPU oracle of the learned coupling-flow variable transform.

TEST INFRASTRUCTURE ONLY: checks the library's flow kernels; nothing in the product
path imports it.

The transform is a RealNVP-style stack of affine coupling layers acting in logit space
of the unit cube (the paper does not use flows; this is the learned alternative to the
periodizing transforms that the library offers beside korobov_r and baker).  For a
cube dimension d, layer l conditions on the coordinates with j % 2 == l % 2 (mask m_l)
and transforms the others:

  MLP_l(v)  = W3 tanh(W2 tanh(W1 v + b1) + b2) + b3,    v = m_l * z   (sizes d, 64, 64, 2d)
  s = 0.25 tanh(o[:d]) * (1 - m_l),   t = o[d:] * (1 - m_l),          o = MLP_l(m_l * z)

  density direction G (x -> u, trained):   z = logit(x);  z <- z exp(s) + t  (l = 0..L-1);
                                            u = sigmoid(z)
      log q(x) = log |det du/dx| = sum_j log(u_j (1 - u_j)) - sum_j log(x_j (1 - x_j))
                                   + sum_l sum_j s_lj
  sampling direction T = G^-1 (u -> x, integrated):
      z = logit(u);  z <- (z - t) exp(-s)  (l = L-1..0);  x = sigmoid(z)
      log J_T(u) = -log q(x)

so the model density of x = T(u), u uniform, is q.  Training maximises the weighted
log-likelihood sum_i w_i log q(x_i) over QMC samples x_i with weights w_i = |W_i f(x_i)|
(the optimum is q proportional to |f|), which needs no derivative of the integrand.  The
integration of a sector with the flow evaluates, per lattice sample y,
u = korobov3(y), x = T(u), weight W = korobov3'(y) J_T(u); a sample with some u_j
outside (0, 1) (rounded to the cube's boundary) contributes 0.

`bf16=True` reproduces the library's arithmetic choices in the network: weights, the
network input and both hidden activations rounded to bfloat16 (round to nearest even,
via float32), products summed exactly in float64 (the library accumulates in float32),
biases and the output in float64; the affine coupling, logit and sigmoid are float64.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64
LAYERS = 4
S_SCALE = 0.25


def bf16(a) -> np.ndarray:
    """Round to bfloat16 (via float32, both round-to-nearest-even); returns float64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def mask(d: int, layer: int) -> np.ndarray:
    return ((np.arange(d) % 2) == (layer % 2)).astype(np.float64)


def init_params(d: int, seed: int = 0, zero_last: bool = True, scale: float = 1.0,
                n_cond: int = 0):
    """Per layer (W1 [64, d + n_cond], b1 [64], W2 [64, 64], b2 [64], W3 [2d, 64], b3 [2d]);
    Glorot-uniform hidden weights, zero biases, and (zero_last) a zero last layer so the
    flow starts as the identity.  All weights are bfloat16 values (stored as float64).
    A conditional flow (n_cond > 0) feeds n_cond conditioning features (kinematic
    invariants of the sector) to every layer's network beside the masked coordinates."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11])))
    params = []
    for _ in range(LAYERS):
        def glorot(o, i):
            lim = scale * np.sqrt(6.0 / (i + o))
            return bf16(rng.uniform(-lim, lim, size=(o, i)))
        W1, W2 = glorot(HIDDEN, d + n_cond), glorot(HIDDEN, HIDDEN)
        W3 = np.zeros((2 * d, HIDDEN)) if zero_last else glorot(2 * d, HIDDEN)
        params.append([W1, np.zeros(HIDDEN), W2, np.zeros(HIDDEN), W3, np.zeros(2 * d)])
    return params


def mlp(p, v, bf=False):
    """o = W3 tanh(W2 tanh(W1 v + b1) + b2) + b3 for rows v [N, d]."""
    W1, b1, W2, b2, W3, b3 = p
    r = bf16 if bf else (lambda a: a)
    h1 = r(np.tanh(r(v) @ r(W1).T + b1))
    h2 = r(np.tanh(h1 @ r(W2).T + b2))
    return h2 @ r(W3).T + b3


def _net_input(z, m, cond):
    v = z * m
    if cond is None:
        return v
    c = np.broadcast_to(np.asarray(cond, dtype=np.float64), (z.shape[0], np.shape(cond)[-1]))
    return np.concatenate([v, c], axis=1)


def _st(p, z, layer, d, bf, cond=None):
    m = mask(d, layer)
    o = mlp(p, _net_input(z, m, cond), bf)
    s = S_SCALE * np.tanh(o[:, :d]) * (1.0 - m)
    t = o[:, d:] * (1.0 - m)
    return s, t


def logit(x):
    return np.log(x) - np.log1p(-x)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def density_direction(params, x, bf=False, cond=None):
    """u = G(x) and log q(x) for rows x [N, d] in (0, 1)^d (conditioning features cond
    [N, c] or [c] for a conditional flow)."""
    x = np.asarray(x, dtype=np.float64)
    d = x.shape[1]
    z = logit(x)
    ssum = np.zeros(x.shape[0])
    for l, p in enumerate(params):
        s, t = _st(p, z, l, d, bf, cond)
        z = z * np.exp(s) + t
        ssum += s.sum(axis=1)
    u = sigmoid(z)
    logq = (np.log(u * (1 - u)).sum(axis=1) - np.log(x * (1 - x)).sum(axis=1) + ssum)
    return u, logq


def sampling_direction(params, u, bf=False, cond=None):
    """x = T(u) and log J_T(u) for rows u [N, d] in (0, 1)^d."""
    u = np.asarray(u, dtype=np.float64)
    d = u.shape[1]
    z = logit(u)
    ssum = np.zeros(u.shape[0])
    for l in reversed(range(len(params))):
        s, t = _st(params[l], z, l, d, bf, cond)
        z = (z - t) * np.exp(-s)
        ssum += s.sum(axis=1)
    x = sigmoid(z)
    logJ = np.log(x * (1 - x)).sum(axis=1) - np.log(u * (1 - u)).sum(axis=1) - ssum
    return x, logJ


def weighted_nll_and_grad(params, x, w, cond=None):
    """Loss L = -sum_i w_i log q(x_i) / sum_i w_i and its gradient with respect to every
    parameter (float64, no bfloat16 rounding), by reverse-mode differentiation with
    torch on the CPU.  Returns (L, grads in the layout of params)."""
    import torch
    tp = [[torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in p] for p in params]
    xt = torch.tensor(np.asarray(x, dtype=np.float64))
    wt = torch.tensor(np.asarray(w, dtype=np.float64))
    d = xt.shape[1]
    z = torch.log(xt) - torch.log1p(-xt)
    ssum = torch.zeros(xt.shape[0], dtype=torch.float64)
    ct = None if cond is None else torch.tensor(
        np.broadcast_to(np.asarray(cond, dtype=np.float64), (xt.shape[0], np.shape(cond)[-1])).copy())
    for l, (W1, b1, W2, b2, W3, b3) in enumerate(tp):
        m = torch.tensor(mask(d, l))
        v = z * m if ct is None else torch.cat([z * m, ct], dim=1)
        h1 = torch.tanh(v @ W1.T + b1)
        h2 = torch.tanh(h1 @ W2.T + b2)
        o = h2 @ W3.T + b3
        s = S_SCALE * torch.tanh(o[:, :d]) * (1 - m)
        t = o[:, d:] * (1 - m)
        z = z * torch.exp(s) + t
        ssum = ssum + s.sum(dim=1)
    u = torch.sigmoid(z)
    logq = (torch.log(u * (1 - u)).sum(dim=1) - torch.log(xt * (1 - xt)).sum(dim=1) + ssum)
    loss = -(wt * logq).sum() / wt.sum()
    loss.backward()
    grads = [[a.grad.numpy().copy() for a in p] for p in tp]
    return float(loss.detach()), grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) of float64 master weights; state = (t, m, v)."""
    t, mom, vel = state
    t += 1
    out_p, out_m, out_v = [], [], []
    for p, g, mp, vp in zip(params, grads, mom, vel):
        lp, lm, lv = [], [], []
        for a, ga, ma, va in zip(p, g, mp, vp):
            ma = b1 * ma + (1 - b1) * ga
            va = b2 * va + (1 - b2) * ga * ga
            mh = ma / (1 - b1 ** t)
            vh = va / (1 - b2 ** t)
            lp.append(a - lr * mh / (np.sqrt(vh) + eps))
            lm.append(ma)
            lv.append(va)
        out_p.append(lp)
        out_m.append(lm)
        out_v.append(lv)
    return out_p, (t, out_m, out_v)


def adam_init(params):
    z = [[np.zeros_like(a) for a in p] for p in params]
    return (0, z, [[np.zeros_like(a) for a in p] for p in params])


def sector_sums(sec, shifts, params, n=None, a=None, bf=True, cond=None, deformed=False):
    """Per-shift estimates of a sector integrated through the flow:
        Q[l, k] = (1/n) sum_i W(y_i) J_T(u_i) f_k(T(u_i)),   u_i = phi(y_i)
    with the sector's periodizing transform phi (weight W) and the flow's sampling
    direction T (conditioned on `cond` for a conditional flow); a sample with a
    coordinate of u or x outside (0, 1) contributes 0.  deformed: f is the integrand on
    the deformed contour, J(x) f(z(x)) (complex).  Lattice points, phi and f come from
    the C oracle; sums are exact (math.fsum, real and imaginary parts separately).
    Returns (Q, S) with S[l, k] = (1/n) sum_i |W J f_k| (tolerance scale)."""
    import math
    from . import integrand, integrand_deformed, korobov_vector, points, transform
    n = int(sec.n if n is None else n)
    z = korobov_vector(n, sec.a if a is None else a, sec.d)
    out = np.empty((len(shifts), sec.K), dtype=np.complex128 if deformed else np.float64)
    scale = np.empty((len(shifts), sec.K))
    for l, sh in enumerate(np.asarray(shifts, dtype=np.float64)):
        y = points(n, z, sh)
        u, w = transform(sec.transform, y)
        W = np.prod(w, axis=1)
        in_u = np.all((u > 0.0) & (u < 1.0), axis=1)
        uu = np.where(in_u[:, None], u, 0.5)
        with np.errstate(divide="ignore"):      # x rounded onto a face: excluded below
            x, logJ = sampling_direction(params, uu, bf, cond)
        in_x = np.all((x > 0.0) & (x < 1.0), axis=1)
        xx = np.where(in_x[:, None], x, 0.5)
        f = integrand_deformed(sec, xx)[0] if deformed else integrand(sec, xx)
        Wt = W * np.exp(logJ)
        use = in_u & in_x & (Wt != 0.0)
        for k in range(sec.K):
            c = np.where(use, Wt * f[:, k], 0.0)
            if deformed:
                out[l, k] = complex(math.fsum(c.real), math.fsum(c.imag)) / n
            else:
                out[l, k] = math.fsum(c) / n
            scale[l, k] = math.fsum(np.abs(c)) / n
    return out, scale


def flatten(params) -> np.ndarray:
    """Parameters in the library's layout: per layer W1, b1, W2, b2, W3, b3 (float32)."""
    return np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for p in params
                           for a in p]).astype(np.float32)


def unflatten(v, d, n_cond=0):
    v = np.asarray(v, dtype=np.float64)
    shapes = [(HIDDEN, d + n_cond), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (2 * d, HIDDEN),
              (2 * d,)]
    out, o = [], 0
    for _ in range(LAYERS):
        layer = []
        for sh in shapes:
            size = int(np.prod(sh))
            layer.append(v[o:o + size].reshape(sh))
            o += size
        out.append(layer)
    return out
