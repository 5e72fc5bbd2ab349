"""Oracle: coefficients of weighted sums given as expressions (arXiv:2305.19768, Sec. 2.4).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Shares no code with the
library's parser and series arithmetic.

The coefficient is parsed with Python's own expression grammar (``ast``, ``^`` read as
``**``), every literal taken from its source text as an exact ``Fraction``; the value
is built as an exact rational function N(eps)/D(eps) with Gaussian-rational
coefficients (no truncation anywhere), and only at the end expanded into a Laurent
series by power-series division of N/eps^vN by D/eps^vD.  That is a different route
from the library's (truncated series arithmetic with tracked precision), so the two
agree only if both are right.

Pins (``tests/test_oracle_coef.py``): geometric and binomial series, the d = 4 - 2 eps
ratio, Laurent poles, complex coefficients, exact decimals, and correct rounding against
``float(Fraction)``.
"""

from __future__ import annotations

import ast
from fractions import Fraction


class G:
    """Gaussian rational re + i im."""

    __slots__ = ("re", "im")

    def __init__(self, re=Fraction(0), im=Fraction(0)):
        self.re = Fraction(re)
        self.im = Fraction(im)

    def __add__(self, o):
        return G(self.re + o.re, self.im + o.im)

    def __sub__(self, o):
        return G(self.re - o.re, self.im - o.im)

    def __mul__(self, o):
        return G(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    def __neg__(self):
        return G(-self.re, -self.im)

    def inv(self):
        n = self.re * self.re + self.im * self.im
        if n == 0:
            raise ZeroDivisionError("division by zero")
        return G(self.re / n, -self.im / n)

    def is_zero(self):
        return self.re == 0 and self.im == 0

    def __repr__(self):
        return f"G({self.re}, {self.im})"


ZERO, ONE = G(0), G(1)


def _trim(p):
    while p and p[-1].is_zero():
        p.pop()
    return p


def padd(a, b):
    n = max(len(a), len(b))
    return _trim([(a[i] if i < len(a) else ZERO) + (b[i] if i < len(b) else ZERO)
                  for i in range(n)])


def pmul(a, b):
    if not a or not b:
        return []
    r = [ZERO] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            r[i + j] = r[i + j] + x * y
    return _trim(r)


class RF:
    """Rational function num(eps) / den(eps); polynomials as coefficient lists."""

    def __init__(self, num, den=None):
        self.num = _trim(list(num))
        self.den = _trim(list(den if den is not None else [ONE]))
        if not self.den:
            raise ZeroDivisionError("division by zero")

    def __add__(self, o):
        return RF(padd(pmul(self.num, o.den), pmul(o.num, self.den)), pmul(self.den, o.den))

    def __neg__(self):
        return RF([-c for c in self.num], self.den)

    def __sub__(self, o):
        return self + (-o)

    def __mul__(self, o):
        return RF(pmul(self.num, o.num), pmul(self.den, o.den))

    def inv(self):
        if not self.num:
            raise ZeroDivisionError("division by zero")
        return RF(self.den, self.num)

    def power(self, e: int):
        base = self if e >= 0 else self.inv()
        r = RF([ONE])
        for _ in range(abs(e)):
            r = r * base
        return r

    def is_constant(self):
        return len(self.num) <= 1 and len(self.den) == 1


def _literal(src: str, node) -> Fraction:
    text = ast.get_source_segment(src, node)
    return Fraction(text)          # exact for integers, decimals and exponent notation


def _build(src: str, node, reg: str, env: dict):
    if isinstance(node, ast.Expression):
        return _build(src, node.body, reg, env)
    if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)) \
            and not isinstance(node.value, bool):
        return RF([G(_literal(src, node))])
    if isinstance(node, ast.Name):
        if node.id == reg:
            return RF([ZERO, ONE])
        if node.id == "I":
            return RF([G(0, 1)])
        if node.id in env:
            return env[node.id]
        raise KeyError(f"no value for symbol {node.id!r}")
    if isinstance(node, ast.UnaryOp) and isinstance(node.op, (ast.USub, ast.UAdd)):
        v = _build(src, node.operand, reg, env)
        return -v if isinstance(node.op, ast.USub) else v
    if isinstance(node, ast.BinOp):
        a = _build(src, node.left, reg, env)
        b = _build(src, node.right, reg, env)
        if isinstance(node.op, ast.Add):
            return a + b
        if isinstance(node.op, ast.Sub):
            return a - b
        if isinstance(node.op, ast.Mult):
            return a * b
        if isinstance(node.op, ast.Div):
            return a * b.inv()
        if isinstance(node.op, ast.Pow):
            if not b.is_constant():
                raise ValueError("exponent depends on the regulator")
            e = b.num[0] * b.den[0].inv() if b.num else ZERO
            if e.im != 0 or e.re.denominator != 1:
                raise ValueError("non-integer exponent")
            return a.power(int(e.re))
    raise ValueError(f"unsupported expression element {ast.dump(node)[:40]}")


def rational_function(expr: str, reg: str = "eps", symbols=None) -> RF:
    """The exact rational function of the coefficient in the regulator."""
    env = {}
    for name, val in (symbols or {}).items():
        s = str(val).replace("^", "**")
        env[name] = _build(s, ast.parse(s, mode="eval"), reg, env)
    s = expr.replace("^", "**")
    return _build(s, ast.parse(s, mode="eval"), reg, env)


def series(expr: str, reg: str = "eps", symbols=None, order_lo: int = 0, n_terms: int = 1):
    """Exact Laurent coefficients: (leading order or None if identically zero,
    [G] coefficients of reg^(order_lo + j), j < n_terms)."""
    f = rational_function(expr, reg, symbols)
    if not f.num:
        return None, [ZERO] * n_terms
    vn = next(i for i, c in enumerate(f.num) if not c.is_zero())
    vd = next(i for i, c in enumerate(f.den) if not c.is_zero())
    a, b = f.num[vn:], f.den[vd:]
    lead = vn - vd
    # power-series division a / b: q_k = (a_k - sum_{j=1..k} b_j q_{k-j}) / b_0
    want = order_lo + n_terms - lead
    q = []
    b0inv = b[0].inv()
    for k in range(max(0, want)):
        acc = a[k] if k < len(a) else ZERO
        for j in range(1, min(k, len(b) - 1) + 1):
            acc = acc - b[j] * q[k - j]
        q.append(acc * b0inv)
    out = []
    for j in range(n_terms):
        k = order_lo + j - lead
        out.append(q[k] if 0 <= k < len(q) else ZERO)
    return lead, out


def to_complex(g: G) -> complex:
    """Nearest doubles of both parts (float(Fraction) rounds correctly)."""
    return complex(float(g.re), float(g.im))
