"""Host checks of the plan-specialised integrand generator (qmc_gen_source /
qmc_specialize with QMC_SPEC_COMPILE_ONLY): no GPU needed.

The generated integrand is straight-line code; these tests interpret it (every line is
a definition by a product, an FMA, a reciprocal, a logarithm or a sum of terms) at
random points of the cube and compare the orders it defines with the oracle's integrand
at the same points, so a wrong factorisation, a dropped monomial, a wrong power or a
misplaced log coefficient fails here.  The compile-only call checks that hiprtc
accepts the generated source for gfx950 at every dimension and precision.
"""
import math
import re

import numpy as np
import pytest

import oracle
import workloads as W


@pytest.fixture(scope="module")
def q():
    import __graft_entry__ as g
    g._ensure_built()
    import paper_2305_19768_amd as qq
    return qq


def _structs(src):
    """{sector: (dtype, body lines)} of the generated source."""
    out = {}
    for m in re.finditer(r"struct G(\d+) \{.*?void (f64|f32)\(.*?for \(int u = 0; u < S; \+\+u\) \{\n(.*?)\n    \}\n",
                         src, flags=re.S):
        out[int(m.group(1))] = (m.group(2), [l.strip() for l in m.group(3).split("\n") if l.strip()])
    return out


def _num(tok):
    tok = tok.strip()
    if tok.endswith("f") and ("0x" in tok or "." in tok):
        tok = tok[:-1]
    if tok.startswith("0x") or tok.startswith("-0x"):
        return float.fromhex(tok)
    return float(tok)


def _interpret(lines, x):
    """Values of the generated definitions at one point x (float64 arithmetic)."""
    env = {}

    def val(tok):
        tok = tok.strip()
        m = re.fullmatch(r"x\[u\]\[(\d+)\]", tok)
        if m:
            return x[int(m.group(1))]
        if tok in env:
            return env[tok]
        return _num(tok)

    def expr(e):
        e = e.strip()
        m = re.fullmatch(r"__builtin_fmaf?\((.*)\)", e)
        if m:
            a, b, c = _split_args(m.group(1))
            return expr(a) * expr(b) + expr(c)
        m = re.fullmatch(r"__builtin_sqrt\((.*)\)", e)
        if m:
            return math.sqrt(expr(m.group(1)))
        m = re.fullmatch(r"\((.*)\) \* (qmc::recip1?\(\w+\)|r)", e)
        if m:
            return expr(m.group(1)) * (1.0 / env["den"])
        m = re.fullmatch(r"qmc::log_(?:f64|pos|tab)\((\w+)(?:, lt)?\)", e)
        if m:
            return math.log(env[m.group(1)])
        m = re.fullmatch(r"__builtin_amdgcn_logf\((\w+)\) \* .*", e)
        if m:
            return math.log(env[m.group(1)])
        if " * " in e:
            v = 1.0
            for t in e.split(" * "):
                v *= expr(t)
            return v
        return val(e)

    for line in lines:
        if line.startswith("float r =") or line.startswith("r = "):
            continue
        m = re.fullmatch(r"(?:const (?:double|float) )?(\w+(?:\[u\]\[\d+\])?) = (.*);", line)
        assert m, line
        name, rhs = m.group(1), m.group(2)
        mm = re.fullmatch(r"f\[u\]\[(\d+)\]", name)
        env[f"f{mm.group(1)}" if mm else name] = expr(rhs)
    return env


def _split_args(s):
    parts, depth, cur = [], 0, ""
    for ch in s:
        if ch == "," and depth == 0:
            parts.append(cur)
            cur = ""
            continue
        depth += ch == "("
        depth -= ch == ")"
        cur += ch
    parts.append(cur)
    return parts


def _check_generated(q, prob, precision, rtol):
    h = q.host_plan(prob, precision=precision)
    try:
        rng = np.random.default_rng(11)
        seen = set()
        for d in sorted({s.d for s in prob.sectors}):
            src = q.gen_source(h, d, f32=precision == q.QMC_PREC_FP32)
            structs = _structs(src)
            for s, (dtype, lines) in structs.items():
                seen.add(s)
                sec = prob.sectors[s]
                for _ in range(4):
                    x = rng.uniform(0.02, 0.98, size=sec.d)
                    env = _interpret(lines, x)
                    f = [env[f"f{k}"] for k in range(sec.K)]
                    ref = oracle.integrand(sec, x[None, :])[0]
                    scale = np.abs(ref).max() + 1e-300
                    assert np.allclose(f, ref, rtol=rtol, atol=rtol * scale), (s, f, ref)
        return seen
    finally:
        q.lib().qmc_plan_free(h)


def test_generated_integrands_match_oracle_two_loop(q):
    prob = W.two_loop_integral(seed=0, n_scale=0.01)
    seen = _check_generated(q, prob, q.QMC_PREC_FP64, 1e-13)
    assert seen == set(range(len(prob.sectors)))   # every sector has code


@pytest.mark.parametrize("d,K,M,u_pow,f_pow2", [(1, 1, 0, 0, -2), (3, 2, 1, -1, -4), (5, 3, 2, 2, -6),
                                                (7, 4, 3, 1, -8), (8, 4, 1, 0, 4), (6, 3, 0, 3, 0),
                                                (2, 4, 3, -2, 2)])
def test_generated_integrand_shapes(q, d, K, M, u_pow, f_pow2):
    rng = np.random.default_rng(7 * d + K)
    ue, uc = W.random_polynomial(rng, d, 6, 2)
    fe, fc = W.random_polynomial(rng, d, 15, 3)
    sec = W.Sector(d=d, u_exp=ue, u_coef=uc, f_exp=fe, f_coef=fc,
                   x_pow2=np.zeros(d, np.int32), u_pow=u_pow, f_pow2=f_pow2,
                   logc=rng.uniform(-1, 1, size=(K, M + 1)), n=20011, a=3, transform="korobov3")
    seen = _check_generated(q, W.single_problem(sec, m=4), q.QMC_PREC_FP64, 1e-13)
    assert seen == {0}


def test_generated_fp32_integrands(q):
    prob = W.two_loop_integral(seed=2, n_sectors=10, n_scale=0.01)
    seen = _check_generated(q, prob, q.QMC_PREC_FP32, 2e-6)
    assert seen   # Euclidean sectors have an FP32 form


def test_repeated_monomials_and_unit_coefficients(q):
    # rows repeated (summed by the planner), a unit coefficient, a pure power x_1^3 and
    # a cancelling pair that leaves a zero coefficient (dropped from the code)
    sec = W.custom_sector(3, u_terms=[(1.0, (0, 0, 0)), (1.0, (1, 0, 0)), (1.0, (0, 1, 0))],
                          f_terms=[(0.5, (0, 0, 0)), (0.25, (3, 0, 0)), (0.125, (1, 1, 1)),
                                   (0.125, (1, 1, 1)), (0.3, (0, 2, 0)), (-0.3, (0, 2, 0)),
                                   (0.7, (0, 0, 2))],
                          u_pow=1, f_pow2=-6, logc=((1.0, 0.0, 0.0), (0.0, -2.0, 0.0),
                                                    (0.0, 0.0, 2.0)), n=1009, a=3,
                          transform="korobov3")
    prob = W.single_problem(sec, m=4)
    assert _check_generated(q, prob, q.QMC_PREC_FP64, 1e-14) == {0}
    h = q.host_plan(prob)
    try:
        src = q.gen_source(h, 3)
    finally:
        q.lib().qmc_plan_free(h)
    body = _structs(src)[0][1]
    ops = [l for l in body if l.startswith("const double t")]
    # at most one operation per variable factor of every non-constant monomial (F: 3 + 3 +
    # 2 after the cancelling x_2^2 pair, U: 1 + 1); the greedy factorisation shares x_1
    assert len(ops) <= 9
    assert "-0x" not in "".join(ops) and "0x1.3333333333333p-2" not in "".join(ops)


def test_one_loop_sector_gets_code(q):
    # x_1^(1/2) U^-1 F^-1 and its log F order: one square root, U F as the denominator
    prob = W.one_loop_sector(seed=0, n=4099, m=4)
    assert _check_generated(q, prob, q.QMC_PREC_FP64, 1e-13) == {0}
    h = q.host_plan(prob)
    try:
        src = q.gen_source(h, 3)
    finally:
        q.lib().qmc_plan_free(h)
    body = _structs(src)[0][1]
    assert "const double hs = __builtin_sqrt(x[u][0]);" in body
    assert "static constexpr bool korobov3 = true;" in src


@pytest.mark.parametrize("transform", ["none", "baker", "korobov1", "korobov3", "korobov6"])
@pytest.mark.parametrize("x_pow2,u_pow,f_pow2", [([1, 0, 3], -2, -3), ([2, -1, 0], 1, 3),
                                                 ([-3, 4, 1], 0, -1), ([0, 0, 0], -1, 5)])
def test_generic_shapes_get_code(q, transform, x_pow2, u_pow, f_pow2):
    # integer and half-integer powers of x_j (positive and negative), half-integer powers
    # of F, every transform, log polynomials of degree above K - 1
    sec = W.custom_sector(3, [(1.0, (0, 0, 0)), (0.5, (1, 0, 0)), (0.25, (0, 1, 1))],
                          [(0.3, (0, 0, 0)), (0.7, (1, 1, 0)), (0.2, (0, 0, 2)), (0.4, (1, 0, 1))],
                          x_pow2=x_pow2, u_pow=u_pow, f_pow2=f_pow2,
                          logc=[[1, 0, 0.5], [0.5, -1, 0]], n=20011, a=5467, transform=transform)
    prob = W.single_problem(sec, m=4, seed=1)
    assert _check_generated(q, prob, q.QMC_PREC_FP64, 1e-13) == {0}
    h = q.host_plan(prob)
    try:
        src = q.gen_source(h, 3)
    finally:
        q.lib().qmc_plan_free(h)
    assert ("static constexpr bool korobov3 = %s;" % ("true" if transform == "korobov3" else "false")) in src
    # a negative power of some x_j makes the integrand infinite on a face of the cube
    neg = any(e < 0 for e in x_pow2)
    assert ("static constexpr bool finite = %s;" % ("false" if neg else "true")) in src


@pytest.mark.slow
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_compile_only_every_dimension(q, precision):
    rng = np.random.default_rng(5)
    secs = [W._two_loop_sector(rng, d, W.next_prime(600 + 97 * d), 0) for d in range(1, 9)]
    prob = W.Problem(sectors=secs, order_lo=-2, m=4,
                     shifts=[W.uniform_shifts(rng, 4, s.d) for s in secs])
    prec = q.QMC_PREC_FP32 if precision == "fp32" else q.QMC_PREC_FP64
    h = q.host_plan(prob, precision=prec)
    try:
        t = q.specialize_compile_only(h)
    finally:
        q.lib().qmc_plan_free(h)
    assert t > 0.0


def test_logarithm_form_follows_the_sign_of_F(q):
    # F with non-negative coefficients and a positive constant is positive on the cube:
    # the generated code takes the table-reduced logarithm without special cases; an F
    # with a negative
    # coefficient keeps the checked form (non-finite sums are then reported)
    logc = [[1, 0, 0], [0, -2, 0], [0, 0, 2]]
    pos = W.custom_sector(3, [(1.0, (0, 0, 0)), (0.5, (1, 0, 0))],
                          [(1.0, (0, 0, 0)), (0.3, (1, 1, 0)), (0.2, (0, 0, 2))], u_pow=1,
                          f_pow2=-6, logc=logc, n=20011, a=5467, transform="korobov3")
    neg = W.custom_sector(3, [(1.0, (0, 0, 0)), (0.5, (1, 0, 0))],
                          [(1.0, (0, 0, 0)), (-0.3, (1, 1, 0)), (0.2, (0, 0, 2))], u_pow=1,
                          f_pow2=-6, logc=logc, n=20011, a=5467, transform="korobov3")
    rng = np.random.default_rng(3)
    prob = W.Problem(sectors=[pos, neg], order_lo=-2, m=4,
                     shifts=[W.uniform_shifts(rng, 4, 3) for _ in range(2)])
    h = q.host_plan(prob)
    try:
        src = q.gen_source(h, 3)
    finally:
        q.lib().qmc_plan_free(h)
    structs = _structs(src)
    body = {s: "\n".join(lines) for s, (_, lines) in structs.items()}
    # finite on the closed cube (no weight-0 test needed) only where F is positive there
    assert "struct G0 {\n  static constexpr bool finite = true;" in src
    assert "struct G1 {\n  static constexpr bool finite = false;" in src
    assert "qmc::log_tab(F, lt)" in body[0] and "qmc::log_f64" not in body[0]
    assert "qmc::log_f64(F)" in body[1] and "qmc::log_tab" not in body[1]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_compile_only_persistent_kernel(q, precision):
    # the batched form's specialised persistent kernel: one program, every sector
    import ctypes
    prob = W.amplitude(seed=1, n_integrals=6, n_sectors=24, d_lo=3, d_hi=6, m=8, n0=1009)
    prec = q.QMC_PREC_FP32 if precision == "fp32" else q.QMC_PREC_FP64
    h = q.host_plan(prob, precision=prec)
    try:
        sec = ctypes.c_double()
        rc = q.lib().qmc_specialize(h, q.QMC_SPEC_COMPILE_ONLY | q.QMC_SPEC_PERSISTENT,
                                    ctypes.byref(sec))
        assert rc == 0, q.lib().qmc_last_error()
        assert sec.value > 0.0
    finally:
        q.lib().qmc_plan_free(h)


def test_persistent_kernel_refuses_other_plans(q):
    import ctypes
    flags = q.QMC_SPEC_COMPILE_ONLY | q.QMC_SPEC_PERSISTENT
    # a complex plan, and a sector outside the batched form's shape (x^(1/2))
    for prob in (W.physical_scan(seed=0, n_points=1, n_sectors=2, d_lo=3, d_hi=4, n=1009, m=16),
                 W.one_loop_sector(seed=0, n=4099, m=4)):
        h = q.host_plan(prob)
        try:
            assert q.lib().qmc_specialize(h, flags, None) == -1
        finally:
            q.lib().qmc_plan_free(h)
    # an FP32 plan with a sector that has no FP32 form
    sec = W.custom_sector(3, [(1.0, (0, 0, 0)), (0.5, (1, 0, 0))],
                          [(1.0, (0, 0, 0)), (-0.3, (1, 1, 0)), (0.2, (0, 0, 2))], u_pow=1,
                          f_pow2=-6, logc=[[1, 0, 0], [0, -2, 0], [0, 0, 2]], n=20011, a=5467,
                          transform="korobov3")
    h = q.host_plan(W.single_problem(sec, m=4), precision=q.QMC_PREC_FP32)
    try:
        assert q.lib().qmc_specialize(h, flags, None) == -1
        assert "FP32" in q.lib().qmc_last_error().decode()
    finally:
        q.lib().qmc_plan_free(h)
