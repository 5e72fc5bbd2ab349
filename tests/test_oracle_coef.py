"""Coefficient expressions (Sec. 2.4): the exact oracle against closed forms, then the
library's parser and series arithmetic (host code behind qmc_coef_series) against the
oracle, bit for bit (both round the same exact rationals to the nearest double)."""
import math
import random
from fractions import Fraction

import pytest

from oracle import coef as OC


def _vals(lead_terms):
    lead, terms = lead_terms
    return lead, [(t.re, t.im) for t in terms]


# ---------------------------------------------------------------- oracle pins
def test_geometric_and_binomial_series():
    lead, t = _vals(OC.series("1/(1-2*eps)", n_terms=8))
    assert lead == 0 and t == [(Fraction(2 ** k), 0) for k in range(8)]
    for n in (1, 2, 3, 5):
        lead, t = _vals(OC.series(f"(1-eps)^(-{n})", n_terms=6))
        assert t == [(Fraction(math.comb(n + k - 1, k)), 0) for k in range(6)]


def test_dimension_ratio_and_poles():
    # d = 4 - 2 eps: (d - 4)/(d - 6) = eps/(1 + eps) = sum_{k>=1} (-1)^(k+1) eps^k
    lead, t = _vals(OC.series("(d-4)/(d-6)", symbols={"d": "4-2*eps"}, n_terms=6))
    assert lead == 1
    assert t == [(Fraction(0), 0)] + [(Fraction((-1) ** (k + 1)), 0) for k in range(1, 6)]
    lead, t = _vals(OC.series("(1+eps)^3/eps^2", order_lo=-2, n_terms=5))
    assert lead == -2 and [r for r, _ in t] == [1, 3, 3, 1, 0]
    lead, t = _vals(OC.series("1/(s-t)", symbols={"s": "3+eps", "t": "3"}, order_lo=-1,
                              n_terms=2))
    assert lead == -1 and [r for r, _ in t] == [1, 0]
    lead, t = _vals(OC.series("((1+eps)^2-1-2*eps)/eps^2", n_terms=2))
    assert lead == 0 and [r for r, _ in t] == [1, 0]
    assert OC.series("eps-eps", n_terms=2)[0] is None


def test_complex_and_exact_literals():
    lead, t = _vals(OC.series("1/(1+I*eps)", n_terms=5))
    want = [(-1j) ** k for k in range(5)]
    assert [complex(r, i) for r, i in t] == want
    assert OC.series("0.1")[1][0].re == Fraction(1, 10)
    assert OC.series("2.5e-3")[1][0].re == Fraction(1, 400)
    assert OC.series("(s+t)/(s*t)", symbols={"s": "3/2", "t": 5})[1][0].re == Fraction(13, 15)


def test_series_agrees_with_direct_evaluation():
    # truncated series at a small eps against plain floating-point evaluation
    rng = random.Random(3)
    for _ in range(20):
        a, b, c = (rng.randint(1, 9) for _ in range(3))
        e = f"({a}+{b}*eps)^2/(({c}-eps)*(1+{a}*eps)) - {b}/({c}+eps)"
        lead, t = OC.series(e, n_terms=12)            # orders 0 .. 11
        assert lead >= 0
        x = 1e-3
        approx = sum(float(v.re) * x ** j for j, v in enumerate(t))
        direct = eval(e.replace("^", "**").replace("eps", repr(x)))
        assert abs(approx - direct) <= 1e-12 * max(1.0, abs(direct)) * 50


# --------------------------------------------------- library against the oracle
@pytest.fixture(scope="module")
def lib():
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2305_19768_amd as q
    return q


def _lib_vs_oracle(q, expr, symbols=None, order_lo=None, n_terms=4):
    olead, oterms = OC.series(expr, symbols=symbols, order_lo=0, n_terms=1)
    llead, _ = q.coef_series(expr, symbols=symbols, order_lo=0, n_terms=0)
    assert llead == olead, (expr, llead, olead)
    if olead is None:
        return
    lo = olead if order_lo is None else order_lo
    _, oterms = OC.series(expr, symbols=symbols, order_lo=lo, n_terms=n_terms)
    _, lterms = q.coef_series(expr, symbols=symbols, order_lo=lo, n_terms=n_terms)
    want = [OC.to_complex(t) for t in oterms]
    assert list(lterms) == want, (expr, list(lterms), want)


def test_library_matches_oracle_on_closed_forms(lib):
    cases = [("1/(1-2*eps)", None), ("(1-eps)^(-3)", None), ("(1+eps)^3/eps^2", None),
             ("(d-4)/(d-6)", {"d": "4-2*eps"}), ("1/(1+I*eps)", None),
             ("(s+t)/(s*t)", {"s": "3/2", "t": "5"}), ("0.1*eps - 2.5e-3", None),
             ("1/((1+eps)^2 - 1)", None), ("((1+eps)^2-1-2*eps)/eps^2", None),
             ("eps - eps", None), ("1/(s-t)", {"s": "3+eps", "t": "3"}),
             ("(2+3*I)/(1-I*eps)^2 + I", None)]
    for e, sym in cases:
        _lib_vs_oracle(lib, e, sym, n_terms=6)


def _random_expr(rng, depth=0):
    if depth > 3 or rng.random() < 0.3:
        return rng.choice(["eps", "s", "t", "u", str(rng.randint(1, 50)),
                           f"{rng.randint(1, 9)}/{rng.randint(1, 9)}", "I", "0.25"])
    op = rng.choice(["+", "-", "*", "/", "^"])
    a = _random_expr(rng, depth + 1)
    if op == "^":
        return f"({a})^{rng.randint(-2, 3)}"
    b = _random_expr(rng, depth + 1)
    if op == "/":
        b = f"({b} + {rng.randint(1, 5)}*eps + {rng.randint(1, 7)})"
    return f"({a}) {op} ({b})"


def test_library_matches_oracle_on_random_rational_functions(lib):
    rng = random.Random(11)
    sym = {"s": "7/3", "t": "-2+eps", "u": "1/(1-eps)"}
    checked = 0
    for _ in range(120):
        e = _random_expr(rng)
        try:
            OC.series(e, symbols=sym, n_terms=1)
        except ZeroDivisionError:
            with pytest.raises(lib.QmcError):
                lib.coef_series(e, symbols=sym, order_lo=-50, n_terms=1)
            continue
        _lib_vs_oracle(lib, e, sym, n_terms=5)
        checked += 1
    assert checked > 80


def test_rounding_to_nearest_double(lib):
    big = 3 ** 200
    cases = [Fraction(2 ** 53 + 1), Fraction(2 ** 53 + 3), Fraction(1, 3), Fraction(-2, 3),
             Fraction(big, big + 1), Fraction(big + 1, 7 ** 90), Fraction(1, 2 ** 1074),
             Fraction(3, 2 ** 1076), Fraction(1, 2 ** 1080), Fraction(5, 2 ** 1075),
             Fraction(2 ** 1023 * 3, 2)]
    rng = random.Random(5)
    for _ in range(200):
        cases.append(Fraction(rng.randint(1, 10 ** rng.randint(1, 60)),
                              rng.randint(1, 10 ** rng.randint(1, 60))))
    for f in cases:
        _, v = lib.coef_series(f"{f.numerator}/{f.denominator}")
        assert v[0].real == float(f) and v[0].imag == 0.0, (f, v[0].real, float(f))


def test_library_errors(lib):
    for e in ["1/(eps-eps)", "2^eps", "sin(eps)", "x+1", "2^(1/2)", "((1", "1 2", "3eps"]:
        with pytest.raises(lib.QmcError):
            lib.coef_series(e, n_terms=1)
    with pytest.raises(lib.QmcError, match="below order_lo"):
        lib.coef_series("1/eps", order_lo=0, n_terms=1)
    assert lib.coef_series("1/eps", order_lo=0, n_terms=0)[0] == -1
    with pytest.raises(lib.QmcError, match="double range"):
        lib.coef_series(f"{2 ** 1100}")


def test_library_survives_malformed_expressions(lib):
    """Token soup, truncated and unbalanced strings, stray bytes: every call returns a
    series or raises QmcError (the parser takes caller strings; under the sanitizer
    build a memory error here aborts the run)."""
    rng = random.Random(2024)
    toks = ["eps", "s", "I", "1", "0", "7", "0.5", "1e3", "2.5e-3", "1e", ".", "e", "+", "-", "*",
            "/", "^", "**", "^-2", "(", ")", "((", "))", " ", "x", "$", "\t", "12345678901234567890",
            "1/0", "eps^-3", ",", "é", "\\", "''", "^^", "--", "**-"]
    accepted = 0
    for _ in range(3000):
        e = "".join(rng.choice(toks) for _ in range(rng.randint(0, 24)))
        if rng.random() < 0.1 and e:
            e = e[:rng.randint(0, len(e))]
        try:
            lead, v = lib.coef_series(e, symbols={"s": "3/2"}, order_lo=-8, n_terms=3)
        except lib.QmcError:
            continue
        accepted += 1
        assert len(v) == 3
    assert accepted > 30
