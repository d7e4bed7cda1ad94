"""The oracle's pins catch plausible mistakes: each case plants one mistake in a copy of the C
oracle (a dropped term, a wrong sign or coefficient, an off-by-one power), builds it, and runs the
pin tests against it; at least one pin must fail.  Nothing here touches the HIP path."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from oracle import build as oracle_build

import test_oracle as pins
import test_oracle_bands as bpins
import test_oracle_moments as mpins
import test_oracle_stream as spins

SRC = oracle_build.SRC

# (name, original text, planted mistake)
MUTANTS = [
    ("sat drops the row above", "if (S) S[y * W + x] = (y > 0 ? S[(y - 1) * W + x] : 0) + run;",
     "if (S) S[y * W + x] = run;"),
    ("sat squares use the pixel", "run_sq += v * v;", "run_sq += v;"),
    ("corner lookup adds the top-left corner with the wrong sign",
     "- sat_at(S, W, y1, x0 - 1) + sat_at(S, W, y0 - 1, x0 - 1);",
     "- sat_at(S, W, y1, x0 - 1) - sat_at(S, W, y0 - 1, x0 - 1);"),
    ("corner lookup drops the left corner", "- sat_at(S, W, y1, x0 - 1) + sat_at(S, W, y0 - 1, x0 - 1);",
     "+ sat_at(S, W, y0 - 1, x0 - 1);"),
    ("variance numerator adds S1^2", "u128 num = (u128)n * sum_sqs[i] - (u128)sums[i] * sums[i];",
     "u128 num = (u128)n * sum_sqs[i] + (u128)sums[i] * sums[i];"),
    ("mean divides by n + 1", "mean[i] = (double)sums[i] / (double)n;", "mean[i] = (double)sums[i] / (double)(n + 1);"),
    ("power tables one power short", "for (int j = 1; j < k; ++j) p *= v;", "for (int j = 2; j < k; ++j) p *= v;"),
    ("skewness with 2 n S1 S2", "const i128 B = N * N * a3 - 3 * N * a1 * a2 + 2 * a1 * a1 * a1;",
     "const i128 B = N * N * a3 - 2 * N * a1 * a2 + 2 * a1 * a1 * a1;"),
    ("skewness without the S1^3 term", "const i128 B = N * N * a3 - 3 * N * a1 * a2 + 2 * a1 * a1 * a1;",
     "const i128 B = N * N * a3 - 3 * N * a1 * a2;"),
    ("kurtosis not in excess", "kurt[i] = A == 0 ? NAN : (double)(C - 3 * A * A) / (a * a);",
     "kurt[i] = A == 0 ? NAN : (double)C / (a * a);"),
    ("kurtosis with 4 n S1^2 S2", "+ 6 * N * a1 * a1 * a2 - 3 * a1 * a1 * a1 * a1;",
     "+ 4 * N * a1 * a1 * a2 - 3 * a1 * a1 * a1 * a1;"),
    ("column totals skip the last row", "for (int64_t y = 0; y < H; ++y) {       /* row by row",
     "for (int64_t y = 0; y < H - 1; ++y) {       /* row by row"),
    ("column totals drop the carry", "T[x] = carry ? carry[x] : 0;", "T[x] = 0;"),
    ("column totals of squares add the pixel", "if (T2) T2[x] += v * v;", "if (T2) T2[x] += v;"),
    ("direct window powers skip the first power", "for (int j = 0; j < k; ++j) {\n                p *= v;\n                sums[j] += p;",
     "for (int j = 0; j < k; ++j) {\n                sums[j] += p;\n                p *= v;"),
    ("resumed stream seeds the row above with the totals, not their running sum",
     "run += carry[x];\n            above[x] = run;", "above[x] = carry[x];"),
    ("resumed stream starts at the window straddling its first row",
     "st->next_k[i] = (r0 + s - 1) / s;", "st->next_k[i] = r0 / s;"),
    ("resumed stream drops the row above in the recurrence",
     "run += st->squares ? v * v : v;\n            cur[x] = (up ? up[x] : 0) + run;",
     "run += st->squares ? v * v : v;\n            cur[x] = run;"),
    ("resumed stream squares use the pixel", "run += st->squares ? v * v : v;", "run += v;"),
    ("resumed stream drops the top-left corner",
     "uint64_t *o = outs[i] + emitted[i] * ow;\n            for (int64_t l = 0; l < ow; ++l) {\n"
     "                int64_t x0 = l * s, x1 = x0 + w - 1;\n"
     "                uint64_t b1 = bot[x1], b0 = x0 > 0 ? bot[x0 - 1] : 0;\n"
     "                uint64_t t1 = top ? top[x1] : 0, t0 = (top && x0 > 0) ? top[x0 - 1] : 0;\n"
     "                o[l] = b1 - t1 - b0 + t0;",
     "uint64_t *o = outs[i] + emitted[i] * ow;\n            for (int64_t l = 0; l < ow; ++l) {\n"
     "                int64_t x0 = l * s, x1 = x0 + w - 1;\n"
     "                uint64_t b1 = bot[x1], b0 = x0 > 0 ? bot[x0 - 1] : 0;\n"
     "                uint64_t t1 = top ? top[x1] : 0, t0 = (top && x0 > 0) ? top[x0 - 1] : 0;\n"
     "                o[l] = b1 - t1 - b0;"),
]

# The pins, called as plain functions with fixed arguments.
PIN_CALLS = [
    (pins.test_golden_worked_example, ()),
    (pins.test_sat_matches_cumsum, (np.uint8,)),
    (pins.test_sat_closed_forms, ()),
    (pins.test_window_sums_match_brute_force_all_windows, ()),
    (pins.test_window_sums_match_numpy_sliding_window, ()),
    (pins.test_mean_std_exact_rationals, ()),
    (pins.test_std_zero_and_binary_windows, ()),
    (mpins.test_power_tables_are_prefix_sums_of_powers, (np.uint8, 256, 4)),
    (mpins.test_window_power_sums_by_corner_lookup_match_direct_sums, ()),
    (mpins.test_moments_match_the_central_definition_in_exact_arithmetic, ()),
    (mpins.test_two_valued_windows_follow_the_bernoulli_closed_forms, (3,)),
    (mpins.test_constant_windows_have_no_shape_and_symmetric_ones_no_skew, ()),
    (bpins.test_column_totals_brute_force, ()),
    (bpins.test_column_totals_are_differences_of_the_last_table_row, (np.uint8,)),
    (bpins.test_band_rows_follow_from_the_band_and_the_totals_above, (np.uint16,)),
    (spins.test_stream_from_any_row_matches_numpy, (np.uint16, True)),
    (spins.test_partition_of_rows_covers_every_output_once, ()),
    (spins.test_stream_wraps_mod_2_64_with_a_large_carry, ()),
]


def failing_pins():
    failed = []
    for fn, args in PIN_CALLS:
        try:
            fn(*args)
        except Exception:        # a failed assertion, or an error the planted mistake provokes
            failed.append(fn.__name__)
    return failed


@pytest.fixture
def use_oracle_library():
    saved = oracle_build.LIB

    def use(path):
        oracle._lib = None
        oracle_build.LIB = path

    yield use
    oracle._lib = None
    oracle_build.LIB = saved


def test_unmutated_oracle_passes_every_pin():
    assert failing_pins() == []


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(name, old, new, use_oracle_library):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation target not found: %s" % name
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "mutant.c")
        lib = os.path.join(d, "mutant.so")
        open(c, "w").write(src.replace(old, new))
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-o", lib, c, "-lm"],
                       check=True)
        use_oracle_library(lib)
        failed = failing_pins()
    assert failed, "no pin catches: %s" % name
