"""Fits the rational approximation of tanh used by the flow network's activations.

tanh(x) ~ x P(x^2) / Q(x^2) on |x| <= XMAX (the argument is clamped there: tanh(9) is
1 - 3e-8, which rounds to the largest float32 below 1), P and Q of degree 4 with P(0) = Q(0) = 1
so that tanh(x) = x exactly in the limit of small x.  The remaining eight coefficients are
fitted by Lawson's iteration (weighted linear least squares whose weights are multiplied
by the current error at every step, converging toward the minimax fit) on the relative
error of P/Q against tanh(x)/x.  Deterministic; prints the float32 coefficients as C
hexadecimal literals and the maximum relative error of the fit in exact arithmetic and
of its float32 evaluation (Horner with fused multiply-adds, one reciprocal).

    python fit_tanh.py
"""
import numpy as np

XMAX = 9.0
DEG = 4


def fit(iters=300):
    x = np.concatenate([XMAX * (1 - np.cos(np.linspace(0, np.pi / 2, 6000))),
                        np.linspace(0, XMAX, 6000)])
    x = np.unique(x[x > 1e-4])
    t = x * x
    g = np.tanh(x) / x
    # unknowns p1..p4, q1..q4:  P(t) - g Q(t) = 0  ->  sum p_k t^k - g sum q_k t^k = g - 1
    A = np.hstack([np.vstack([t ** k for k in range(1, DEG + 1)]).T,
                   -(g[:, None] * np.vstack([t ** k for k in range(1, DEG + 1)]).T)])
    b = g - 1.0
    w = np.ones_like(x)
    Q = np.ones_like(x)
    best = None
    for _ in range(iters):
        W = np.sqrt(w) / (Q * g)           # relative error of P/Q, linearised at the last Q
        c, *_ = np.linalg.lstsq(A * W[:, None], b * W, rcond=None)
        p = np.concatenate([[1.0], c[:DEG]])
        q = np.concatenate([[1.0], c[DEG:]])
        P = np.polyval(p[::-1], t)
        Q = np.polyval(q[::-1], t)
        err = np.abs(P / Q / g - 1.0)
        if best is None or err.max() < best[2]:
            best = (p, q, err.max())
        w = w * err / err.mean()
        w /= w.mean()
    return best


def eval_f32(p, q, xs):
    """x P(x^2) / Q(x^2) as the kernel evaluates it: clamp, fused Horner steps rounded to
    float32, the product with x, one reciprocal, one product."""
    f32 = np.float32
    c = np.clip(xs.astype(f32), f32(-XMAX), f32(XMAX))
    t = (c.astype(np.float64) ** 2).astype(f32)

    def horner(cs):
        acc = np.full_like(t, f32(cs[-1]))
        for k in range(len(cs) - 2, -1, -1):
            acc = (acc.astype(np.float64) * t + np.float64(f32(cs[k]))).astype(f32)
        return acc

    num = (c.astype(np.float64) * horner(p)).astype(f32)
    rq = (1.0 / horner(q).astype(np.float64)).astype(f32)
    return (num.astype(np.float64) * rq).astype(f32)


if __name__ == "__main__":
    p, q, e = fit()
    pf = [float(np.float32(v)) for v in p]
    qf = [float(np.float32(v)) for v in q]
    xs = np.concatenate([np.linspace(-12, 12, 2000001),
                         np.geomspace(1e-30, 12, 200001), -np.geomspace(1e-30, 12, 200001)])
    r = eval_f32(pf, qf, xs)
    ref = np.tanh(xs.astype(np.float32).astype(np.float64))
    nz = ref != 0
    rel = np.abs(r[nz] / ref[nz] - 1.0)
    print("P:", ", ".join(float(v).hex() for v in pf))
    print("Q:", ", ".join(float(v).hex() for v in qf))
    print(f"max relative error: fit {e:.3e}, float32 evaluation {rel.max():.3e} "
          f"(median {np.median(rel):.2e})")
