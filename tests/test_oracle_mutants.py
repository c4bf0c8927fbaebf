"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a private copy of the oracle's C source (on
the CPU, never in the GPU library), builds it, and runs the pin checks of
test_oracle_pins.py against it: at least one check must fail.  This shows the
pins are sensitive to a dropped term, a wrong sign or index, a wrong tie rule,
a wrong summation order, a wrong empty-cluster rule and unsound pruning.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle
import tests.test_oracle_exact_mean as xm
import tests.test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "knor_oracle.c")

# (name, exact text in the source, replacement)
MUTANTS = [
    ("sign", "double t = x[i] - c[i];", "double t = x[i] + c[i];"),
    ("dropped-dim", "for (int i = 0; i < d; ++i) {\n    double t",
     "for (int i = 0; i < d - 1; ++i) {\n    double t"),
    ("tie-rule", "if (D < best) { best = D; a = j; }",
     "if (D <= best) { best = D; a = j; }"),
    ("count-off-by-one", "double dn = (double)nj;", "double dn = (double)(nj + 1);"),
    ("empty-to-zero",
     "memcpy(c, C_prev + (size_t)j * d, sizeof(double) * (size_t)d);",
     "memset(c, 0, sizeof(double) * (size_t)d);"),
    ("tree-split", "while (h * 2 < m) h *= 2;", "while (h * 2 <= m - 1 && h < 2) h *= 2;"),
    ("leaf-double-count", "for (int64_t m = m0 + 1; m < m1; ++m) {\n      const double* x",
     "for (int64_t m = m0; m < m1; ++m) {\n      const double* x"),
    ("row-index", "const double* x = X + (size_t)idx[m] * d;",
     "const double* x = X + (size_t)idx[m];"),
    ("no-half", "s[i] = 0.5 * m;\n      }\n      for (int64_t p",
     "s[i] = m;\n      }\n      for (int64_t p"),
    ("no-drift", "for (int64_t p = 0; p < n; ++p) u[p] = u[p] + drift[a[p]];",
     "for (int64_t p = 0; p < n; ++p) u[p] = u[p];"),
    ("exact-ties-away", "if (round && (sticky || (mant & 1u))) mant += 1;",
     "if (round) mant += 1;"),
    ("exact-truncate", "if (round && (sticky || (mant & 1u))) mant += 1;", ""),
    ("exact-sign-lost", "xw_add_shifted(v > 0 ? a->pos : a->neg, m, shift);",
     "xw_add_shifted(a->pos, m, shift);"),
    ("exact-carry-dropped", "    carry = c1 | c2;\n", "    carry = 0;\n"),
    ("exact-unit", "int64_t shift = (int64_t)e - 53 + 1074;",
     "int64_t shift = (int64_t)e - 52 + 1074;"),
    ("exact-subnormal-lost", "m >>= -shift;", "m = 0;"),
    ("exact-empty-to-zero",
     "for (int i = 0; i < d; ++i) c[i] = C_prev[(size_t)j * d + i];",
     "for (int i = 0; i < d; ++i) c[i] = 0.0;"),
    ("clause2-no-half", "0.5 * CC[(size_t)a * k + j] * (1.0 - ETA)) continue;\n    if",
     "1.0 * CC[(size_t)a * k + j] * (1.0 - ETA)) continue;\n    if"),
    ("objective-wrong-centroid",
     "D[p] = oracle_dist2(X + (size_t)p * d, C + (size_t)labels[p] * d, d);",
     "D[p] = oracle_dist2(X + (size_t)p * d, C, d);"),
    ("objective-plain-order",
     "double s = oracle_canonical_sum(D, n);\n  free(D);",
     "double s = 0.0;\n  for (int64_t p = 0; p < n; ++p) s += D[p];\n  free(D);"),
]

CHECKS = [
    (pins.test_golden_2d_integer_assign_update_fit, {}),
    (pins.test_golden_1d_threshold, {}),
    (pins.test_objective_golden_2d_integer, {}),
    (pins.test_objective_summation_order_golden, {}),
    (pins.test_objective_bruteforce_integer, {"seed": 0}),
    (pins.test_golden_canonical_order, {}),
    (pins.test_dist2_integer_exact, {}),
    (pins.test_tie_lowest_index, {}),
    (pins.test_bruteforce_fixed_point_and_optimum, {"seed": 0}),
    (pins.test_bruteforce_fixed_point_and_optimum, {"seed": 3}),
    (pins.test_k_equals_one_is_global_mean, {}),
    (pins.test_empty_cluster_keeps_previous, {}),
    (pins.test_objective_nonincreasing_and_means, {"seed": 0}),
    (pins.test_canonical_sum_bottom_up, {"m": 300}),
    (pins.test_canonical_sum_bottom_up, {"m": 4097}),
    (pins.test_mti_equals_plain_every_iteration, {"case": "cfg2"}),
    (pins.test_mti_equals_plain_every_iteration, {"case": "uniform"}),
    (pins.test_mti_equals_plain_every_iteration, {"case": "dups"}),
    (xm.test_exact_mean_is_correctly_rounded, {"seed": 0}),
    (xm.test_exact_mean_ties_to_even, {}),
    (xm.test_exact_mean_subnormal_and_extreme, {}),
    (xm.test_exact_mean_many_terms_carry, {}),
    (xm.test_update_exact_against_rationals, {"seed": 0}),
]


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(workdir, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique/found"
    mut = src.replace(old, new)
    cpath = os.path.join(workdir, f"{name}.c")
    spath = os.path.join(workdir, f"lib{name}.so")
    with open(cpath, "w") as f:
        f.write(mut)
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", spath, cpath, "-lm"])
    orc = oracle.Oracle(spath)
    failed = []
    for fn, kw in CHECKS:
        try:
            fn(orc, **kw)
        except Exception as e:   # an assertion, or a crash-free error path
            failed.append((fn.__name__, type(e).__name__))
    print(name, failed)
    assert failed, f"no pin caught mutant {name}"
