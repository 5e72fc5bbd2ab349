"""Planted mistakes in the oracle: every mutant must fail at least one pin.

A mutant is the oracle's own source with one textual change of the kind the pins exist
to catch: a dropped term, a wrong power, index, sign or branch.  Python mutants
(``oracle/__init__.py``, ``oracle/flow.py``) are executed from the modified text and
replace the functions of the module for the duration of one check; C mutants
(``oracle/qmc_oracle.c``) are compiled into a temporary library that the package loads
in place of its own.  The pins are the test functions of the pin modules, called
unchanged: each must fail on its mutant, by an assertion or by the oracle's own error
report (and passes on the real oracle, where it is collected in its own module).  Every
planted change must match the source exactly once, so a refactoring of the oracle that
removes a site fails here loudly instead of silently weakening the check.
"""
import inspect

import pytest

import oracle
import oracle.flow as oracle_flow
from oracle import build as oracle_build

import test_oracle_adaptive as TA
import test_oracle_deform as TD
import test_oracle_flow as TF
import test_oracle_pins as TP

def _mutated(path, old, new):
    with open(path) as fh:
        src = fh.read()
    assert src.count(old) == 1, f"planted site {old!r} occurs {src.count(old)} times in {path}"
    return src.replace(old, new)


def _python_mutant(monkeypatch, module, old, new):
    src = _mutated(module.__file__, old, new)
    ns = {"__name__": module.__name__, "__file__": module.__file__,
          "__package__": module.__package__}
    exec(compile(src, module.__file__ + " (mutant)", "exec"), ns)
    for name, val in ns.items():
        if inspect.isfunction(val) and inspect.isfunction(getattr(module, name, None)):
            monkeypatch.setattr(module, name, val)


def _c_mutant(monkeypatch, tmp_path, old, new):
    src = _mutated(oracle_build.SRC, old, new)
    path = tmp_path / "qmc_oracle_mutant.c"
    path.write_text(src)
    lib = oracle_build.compile_lib(str(path), str(tmp_path / "libqmc_oracle_mutant.so"))
    monkeypatch.setattr(oracle, "_LIB_PATH", lib)
    monkeypatch.setattr(oracle, "_lib", None)


# A pin fails by an assertion or by the oracle's own error report (a non-finite sample
# or a contour that no deformation parameter makes valid).
PIN_FAILURES = (AssertionError, oracle.OracleNonFinite, oracle.OracleSignCheck)


def _fails_a_pin(pins):
    caught = []
    for pin in pins:
        try:
            pin()
        except PIN_FAILURES:
            caught.append(getattr(pin, "__name__", repr(pin)))
    return caught


def _p(fn, *args):
    def run():
        return fn(*args)
    run.__name__ = f"{fn.__name__}{args if args else ''}"
    return run


ALLOC = [_p(TA.check_allocation_round_properties, oracle)]

# (name, file, old, new, pins)
MUTANTS = [
    # --- adaptive weighted sums (Sec. 2.1.3)
    ("error not squared in w", "py", "err[s, k - p] ** 2", "err[s, k - p]", ALLOC),
    ("order offset of the series term dropped", "py", "err[s, k - p] ** 2", "err[s, k] ** 2",
     ALLOC),
    ("integral variance in place of the sector's", "py", "err[s, k - p] ** 2",
     "ierr[problem.sectors[s].integral, k - p] ** 2", ALLOC),
    ("w without n^alpha", "py", "* n_cur[s] ** alpha", "* n_cur[s]", ALLOC),
    ("|c| in place of |c|^2", "py", "abs(ci[p]) ** 2", "abs(ci[p])", ALLOC),
    ("closed form without the alpha factor", "py", "n = (alpha * w * lam * c2 / tau)",
     "n = (w * lam * c2 / tau)",
     [TP.test_allocation_satisfies_constraint_and_stationarity,
      TP.test_allocation_is_the_constrained_minimum] + ALLOC),
    ("series variance with the wrong order", "py",
     "vre[j] += c.real ** 2 * er[i, j - p] ** 2", "vre[j] += c.real ** 2 * er[i, j] ** 2",
     [TP.test_amplitude_series_is_the_product_of_series]),
    ("variance with m instead of m - 1", "py", "var = ((Q - mean) ** 2).sum(axis=0) / (m - 1)",
     "var = ((Q - mean) ** 2).sum(axis=0) / m", [TP.test_estimate_is_mean_and_standard_error]),
    ("amplitude variance without Im C", "py",
     "var_re = (cr ** 2 * er ** 2 + ci ** 2 * ei ** 2).sum(axis=0)",
     "var_re = (cr ** 2 * er ** 2).sum(axis=0)",
     [TP.test_amplitude_variance_propagation_and_eps_rel]),
    # --- lattice rule, transforms, integrand, sums (C)
    ("shift not applied", "c", "double v = q + delta[j];", "double v = q;",
     [TP.test_lattice_rule_aliases_predicted_dual_vectors,
      TP.test_lattice_quotient_is_ieee_and_shift_wraps_exactly]),
    ("wrong modulus", "c", "uint64_t k = mulmod(i, z[j], n);",
     "uint64_t k = mulmod(i, z[j], n - 1);",
     [_p(TP.test_lattice_columns_are_permutations, 101, 12),
      TP.test_lattice_rule_exact_on_trig_polynomials]),
    ("korobov density without its normalisation", "c",
     "double dens = (double)N * binom(2 * r, r)", "double dens = binom(2 * r, r)",
     [_p(TP.test_korobov_transform_properties, "korobov3", 3)]),
    ("monomial exponents transposed", "c", "v *= ipow(x[j], exps[t * d + j]);",
     "v *= ipow(x[j], exps[t * d + (d - 1 - j)]);",
     [TP.test_mixed_monomial_exponents_not_transposed,
      _p(TP.test_massless_box_six_dimensions_closed_form, 3.7, 1.3)]),
    ("half-integer power of F as an integer power", "c",
     "base *= pow(F, 0.5 * (double)g->f_pow2);", "base *= pow(F, (double)(g->f_pow2 / 2));",
     [_p(TP.test_closed_form_integrals, "F^-1/2")]),
    ("log powers reversed", "c", "s += g->logc[k * (g->M + 1) + m] * ipow(L, m);",
     "s += g->logc[k * (g->M + 1) + m] * ipow(L, g->M - m);", [TP.test_bubble_log_moments]),
    ("power of U dropped", "c", "base *= pow(U, (double)g->u_pow);", "base *= 1.0;",
     [_p(TP.test_massless_box_six_dimensions_closed_form, 1.0, 1.0)]),
    ("zero-weight samples evaluated", "c",
     "if (W == 0.0)\n                continue;\n            integrand(&g, x, fk);",
     "if (W != W)\n                continue;\n            integrand(&g, x, fk);",
     [TP.test_zero_weight_samples_are_skipped_and_nonfinite_is_reported]),
    ("compensation dropped", "c", "a->c += (a->s - t) + v;", "a->c += 0.0 * ((a->s - t) + v);",
     [TP.test_neumaier_sum_is_compensated]),
    ("B_2 constant", "c", "double b2 = x * x - x + 1.0 / 6.0;",
     "double b2 = x * x - x + 1.0 / 3.0;", [TP.test_p2_equals_dual_lattice_series]),
    # --- contour deformation (C)
    ("Hessian term of the Jacobian dropped", "c",
     "A[j * d + k] = -I * (lambda * s * H[j * d + k]);", "A[j * d + k] = 0.0;",
     [TD.test_cauchy_invariance_two_dimensional, TD.test_jacobian_and_map_against_definitions]),
    ("diagonal term of the Jacobian dropped", "c",
     "A[j * d + j] += 1.0 - I * (lambda * (1.0 - 2.0 * x[j]) * grad[j]);",
     "A[j * d + j] += 1.0;",
     [TD.test_cauchy_invariance_two_dimensional, TD.test_jacobian_and_map_against_definitions]),
    ("deformation with the wrong sign", "c", "z[j] = x[j] - I * (lambda * s * grad[j]);",
     "z[j] = x[j] + I * (lambda * s * grad[j]);",
     [_p(TD.test_bubble_above_threshold_closed_form, "inverse"),
      TD.test_jacobian_and_map_against_definitions]),
    ("gradient without the exponent factor", "c", "double v = coef[t] * (double)e[j];",
     "double v = coef[t];", [TD.test_jacobian_and_map_against_definitions]),
    ("+i0 branch on the negative axis", "c", "arg = -M_PI;", "arg = M_PI;",
     [TD.test_branch_of_f_minus_i0_on_the_real_contour]),
    ("U left on the real contour", "c",
     "cplx U = cpoly(g->d, g->n_u, g->u_exp, g->u_coef, z);",
     "cplx U = creal(cpoly(g->d, g->n_u, g->u_exp, g->u_coef, z));",
     [_p(TD.test_cauchy_invariance_monomial_and_u, "u_power")]),
    # --- learned flow transform (Python)
    ("sign of s in log q", "flow", "- np.log(x * (1 - x)).sum(axis=1) + ssum)",
     "- np.log(x * (1 - x)).sum(axis=1) - ssum)",
     [_p(TF.test_invertibility_and_logdet_cancel, 5), TF.test_logdet_against_finite_differences]),
    ("logit Jacobian dropped in the sampling direction", "flow",
     "logJ = np.log(x * (1 - x)).sum(axis=1) - np.log(u * (1 - u)).sum(axis=1) - ssum",
     "logJ = -ssum", [TF.test_transformed_integral_is_unbiased]),
    ("layers inverted in the wrong order", "flow", "for l in reversed(range(len(params))):",
     "for l in range(len(params)):", [_p(TF.test_invertibility_and_logdet_cancel, 5)]),
    ("affine coupling inverted wrongly", "flow", "z = (z - t) * np.exp(-s)",
     "z = z * np.exp(-s) - t", [_p(TF.test_invertibility_and_logdet_cancel, 5)]),
    ("Adam without bias correction", "flow", "mh = ma / (1 - b1 ** t)", "mh = ma",
     [TF.test_first_adam_step_closed_form]),
]


@pytest.mark.parametrize("name,where,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(monkeypatch, tmp_path, name, where, old, new, pins):
    if where == "py":
        _python_mutant(monkeypatch, oracle, old, new)
    elif where == "flow":
        _python_mutant(monkeypatch, oracle_flow, old, new)
    else:
        _c_mutant(monkeypatch, tmp_path, old, new)
    caught = _fails_a_pin(pins)
    assert caught, f"mutant '{name}' passed every pin in {[getattr(p, '__name__', p) for p in pins]}"
