"""Each plausible mistake planted in a copy of the oracle's C source (a
flipped sign, a dropped factor, a wrong threshold or index) must make at
least one of the oracle pins fail.  The mutants are compiled and run on the
CPU only."""
import os

import pytest

import oracle
from tests import test_oracle_gumbel as Gp
from tests import test_oracle_pins as P
from tests.conftest import read_golden

MUTANTS = {
    "negation_swapped": ("return (code & 1) ? xv : 1.0 - xv;", "return (code & 1) ? 1.0 - xv : xv;"),
    "slope_sign": ("return (code & 1) ? 1.0 : -1.0;", "return (code & 1) ? -1.0 : 1.0;"),
    "dropped_right_product": ("const double others = left[j] * right;", "const double others = left[j];"),
    "right_not_advanced": ("right *= a[j];", "right *= 1.0;"),
    "round_tie_to_one": ("const int value = xr[code >> 1] > 0.5;", "const int value = xr[code >> 1] >= 0.5;"),
    "unsat_inverted": ("if (!any_true) ++cnt;", "if (any_true) ++cnt;"),
    "best_tie_last": ("if (unsat[(int64_t)f * R + r] < unsat[(int64_t)f * R + b]) b = r;",
                      "if (unsat[(int64_t)f * R + r] <= unsat[(int64_t)f * R + b]) b = r;"),
    "loss_transposed": ("if (loss) loss[(int64_t)f * R + r] = s;", "if (loss) loss[(int64_t)r * F + f] = s;"),
    "adam_no_bias_correction": ("double y = x[i] - lr * (mom[i] / c1)", "double y = x[i] - lr * (mom[i])"),
    "gumbel_tie_to_one": ("xh[i] = s > 0.0f ? 1.0 : 0.0;", "xh[i] = s >= 0.0f ? 1.0 : 0.0;"),
    "gumbel_single_logit_step": ("d[i] -= 2.0 * lr * g1;", "d[i] -= lr * g1;"),
    "gumbel_no_temperature": ("const double g1 = G[i] * y1 * (1.0 - y1) / tau;",
                              "const double g1 = G[i] * y1 * (1.0 - y1);"),
    "gumbel_wrong_sigmoid": ("const double y1 = 1.0 / (1.0 + exp(-(d[i] + (double)l[i]) / tau));",
                             "const double y1 = 1.0 / (1.0 + exp(-(d[i] - (double)l[i]) / tau));"),
    "sgd_no_upper_clamp": ("    if (y > 1.0) y = 1.0;\n    x[i] = y;\n  }\n}\n\n/* Adam",
                           "    x[i] = y;\n  }\n}\n\n/* Adam"),
    "def_mode_includes_self": ("if (i != j) others *= factor(c[i], xr);", "others *= factor(c[i], xr);"),
    "full_step_counts_after_update": (
        "  oracle_unsat(n, F, fcb, cptr, lits, R, x, unsat);\n  oracle_grad(n, F, fcb, cptr, lits, R, x, loss, grad, NULL);\n  oracle_step_sgd((int64_t)R * n, lr, x, grad);",
        "  oracle_grad(n, F, fcb, cptr, lits, R, x, loss, grad, NULL);\n  oracle_step_sgd((int64_t)R * n, lr, x, grad);\n  oracle_unsat(n, F, fcb, cptr, lits, R, x, unsat);"),
    "full_step_half_rate": ("oracle_step_sgd((int64_t)R * n, lr, x, grad);\n}",
                            "oracle_step_sgd((int64_t)R * n, 0.5 * lr, x, grad);\n}"),
    "empty_product_zero": ("  double u = 1.0;\n  for (int32_t i = 0; i < k; ++i) u *= factor",
                           "  double u = (k == 0) ? 0.0 : 1.0;\n  for (int32_t i = 0; i < k; ++i) u *= factor"),
}


def _pins():
    g = read_golden
    return [
        lambda: P.test_eq1_or_not_and_polynomials(),
        lambda: P.test_eq2_brute_force_all_assignments(0),
        lambda: P.test_empty_clause_always_unsat(),
        lambda: P.test_golden_intro_example(g),
        lambda: P.test_golden_appendix_normalization(g, "clauses", 0.0),
        lambda: P.test_loss_is_expected_unsat_count(3),
        lambda: P.test_gradient_flip_identity(),
        lambda: P.test_gradient_matches_autograd_with_repeats(5),
        lambda: P.test_zero_safe_partials(),
        lambda: P.test_sgd_step_matches_torch_optim(),
        lambda: P.test_adam_steps_match_torch_optim(),
        lambda: P.test_unsat_count_with_ties_at_half(),
        lambda: P.test_best_is_first_minimum(),
        lambda: P.test_batch_equals_formulas_alone(),
        lambda: P.test_full_step_matches_autograd_sgd_and_boolean_count(),
        lambda: Gp.test_step_matches_two_logit_autograd(True, 1.0),
        lambda: Gp.test_step_matches_two_logit_autograd(False, 0.5),
        lambda: Gp.test_tie_goes_to_state_zero(),
    ]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = oracle.source()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    lib = oracle.build_variant(src.replace(old, new), os.path.join(str(tmp_path), f"mut_{name}.so"))
    failures = 0
    with oracle.use_library(lib):
        for pin in _pins():
            try:
                pin()
            except AssertionError:
                failures += 1
    assert failures >= 1, f"no pin detects the mutant {name}"
