"""Each plausible slip planted in a copy of the oracle trips at least one pin.

The mutants are built on the CPU from the oracle's source with one textual
change each (a dropped term, a wrong sign, transposed operands, an off-by-one
grid index, ...).  This shows that the pins in oracle_pins.py constrain every
part of the oracle's arithmetic, not just its overall shape.
"""
import os

import pytest

import oracle
from gen_pins import GEN_PINS
from oracle_pins import ALL_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "lsp_oracle.c")

MUTANTS = {
    "dropped_sine_term": ("p += YS * YS / SS;", "p += 0.0;"),
    "dropped_cosine_term": ("p += YC * YC / CC;", "p += 0.0;"),
    "wrong_sign_shift": ("long double a = w * ((long double)t - shift);",
                         "long double a = w * ((long double)t + shift);"),
    "tau_missing_factor_two": ("ora_sum_get(&sc)) / (2.0L * w);", "ora_sum_get(&sc)) / w;"),
    "atan2_transposed": ("atan2(ora_sum_get(&ss), ora_sum_get(&sc))",
                         "atan2(ora_sum_get(&sc), ora_sum_get(&ss))"),
    "grid_off_by_one": ("return f_min + df * (double)i;", "return f_min + df * (double)(i + 1);"),
    "grid_closed_interval": ("double df = (f_max - f_min) / (double)n_f;",
                             "double df = (f_max - f_min) / (double)(n_f - 1);"),
    "mean_not_removed": ("ybar = ora_sum_get(&sy) / (double)n;", "ybar = 0.0;"),
    "normalisation_missing_two": ("return 2.0 * pls / syy;", "return pls / syy;"),
    "omega_missing_two_pi": ("return ORA_TWO_PI * f;", "return f;"),
    "argmax_last_tie": ("if (best < 0 || p[i] > bp) {", "if (best < 0 || p[i] >= bp) {"),
    "cos_denominator_from_sine": ("ora_sum_add(&cc, c * c);", "ora_sum_add(&cc, s * s);"),
    "swapped_numerators": ("ora_sum_add(&yc, yp[j] * c);", "ora_sum_add(&yc, yp[j] * s);"),
    "no_degenerate_term_rule": ("if (SS > 1e-12 * (double)n)", "if (1)"),
    "period_missing_two_pi": ("return ORA_TWO_PI / ora_omega(f, unit);",
                              "return 1.0 / ora_omega(f, unit);"),
    "window_single_angle": ("ora_sincos(2.0L * w, t[j], 0.0L, &s2, &c2);",
                            "ora_sincos(w, t[j], 0.0L, &s2, &c2);"),
}

# Slips in the generalized periodogram (Section 4.11), caught by its own pins.
GEN_MUTANTS = {
    "gen_mean_not_floated": ("ybar = ora_sum_get(&swy) / *wsum;", "ybar = 0.0;"),
    "gen_weights_not_squared": ("w[j] = dy ? 1.0 / (dy[j] * dy[j]) : 1.0;",
                                "w[j] = dy ? 1.0 / dy[j] : 1.0;"),
    "gen_error_check_missing": ("if (dy && !(isfinite(dy[j]) && dy[j] > 0.0))", "if (0)"),
    "gen_yy_unweighted": ("ora_sum_add(&sq, w[j] * yw[j] * yw[j]);",
                          "ora_sum_add(&sq, yw[j] * yw[j]);"),
    "gen_means_unweighted": ("ora_sum_add(&c, w[j] * cj);", "ora_sum_add(&c, cj);"),
    "gen_tau_not_centred": ("ora_sincos(om, t[j], 0.0L, &sj, &cj);\n        dc = cj - mc;",
                            "ora_sincos(om, t[j], 0.0L, &sj, &cj);\n        dc = cj;"),
    "gen_tau_transposed": ("atan2(2.0 * ora_sum_get(&cs), ora_sum_get(&cc) - ora_sum_get(&ss))",
                           "atan2(ora_sum_get(&cc) - ora_sum_get(&ss), 2.0 * ora_sum_get(&cs))"),
    "gen_tau_missing_two": ("ora_sum_get(&ss)) /\n           (2.0L * om);",
                            "ora_sum_get(&ss)) /\n           om;"),
    "gen_wrong_sign_shift": ("long double a = w * ((long double)t - shift);",
                             "long double a = w * ((long double)t + shift);"),
    "gen_shift_not_centred": ("ora_sincos(om, t[j], tau, &sj, &cj);\n        dc = cj - mc;\n"
                              "        ds = sj - ms;",
                              "ora_sincos(om, t[j], tau, &sj, &cj);\n        dc = cj - mc;\n"
                              "        ds = sj;"),
    "gen_numerator_unweighted": ("ora_sum_add(&yc, w[j] * yw[j] * dc);",
                                 "ora_sum_add(&yc, yw[j] * dc);"),
    "gen_denominator_from_sine": ("w[j] * yw[j] * ds);\n        ora_sum_add(&cc, w[j] * dc * dc);",
                                  "w[j] * yw[j] * ds);\n        ora_sum_add(&cc, w[j] * ds * ds);"),
    "gen_dropped_sine_term": ("p += gs * gs / gss;", "p += 0.0;"),
    "gen_no_drop_rule": ("if (gss > 1e-12 * wsum)", "if (1)"),
    "gen_normalisation_missing_two": ("return 2.0 * pls / yy;", "return pls / yy;"),
}


def _caught(name, old, new, pins, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = oracle.compile_source(str(path), str(tmp_path / "libmutant.so"))
    ora = oracle.Oracle(lib)
    caught = []
    for pin in pins:
        try:
            pin(ora)
        except AssertionError:
            caught.append(pin.__name__)
    return caught


@pytest.mark.parametrize("name", sorted(GEN_MUTANTS))
def test_gen_mutant_is_caught(name, tmp_path):
    old, new = GEN_MUTANTS[name]
    assert _caught(name, old, new, GEN_PINS, tmp_path), f"no pin catches mutant {name}"


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = oracle.compile_source(str(path), str(tmp_path / "libmutant.so"))
    ora = oracle.Oracle(lib)
    caught = []
    for pin in ALL_PINS:
        try:
            pin(ora)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"no pin catches mutant {name}"
