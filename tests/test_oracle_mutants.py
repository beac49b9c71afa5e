"""Each plausible mistake planted in a copy of the oracle must fail a pin.

The mutants are built from the oracle's source by a single textual
substitution, compiled into a temporary directory with the same flags, and
checked in a subprocess (a planted mistake may crash or loop; the
subprocess has a time limit).  All of this runs on the CPU.
"""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, text in prop_oracle.c, replacement)
MUTANTS = [
    ("min_act_picks_wrong_bound",
     "    double bmin = a > 0.0 ? L[j] : U[j];\n    double bmax = a > 0.0 ? U[j] : L[j];\n    if (isinf(bmin)) cmin++;",
     "    double bmin = a > 0.0 ? U[j] : L[j];\n    double bmax = a > 0.0 ? L[j] : U[j];\n    if (isinf(bmin)) cmin++;"),
    ("dropped_plus_b_term", "    t = t / a;\n    t = t + b;\n", "    t = t / a;\n"),
    ("beta_minus_sign_flipped", "  if (act_inf == 0) {\n    t = beta - act_fin;",
     "  if (act_inf == 0) {\n    t = act_fin - beta;"),
    ("negative_coef_sides_swapped",
     "        if (has_min) { lc_raw = tmin; has_l = 1; }\n        if (has_max) { uc_raw = tmax; has_u = 1; }\n      }\n      if (has_l && lower_counts",
     "        if (has_min) { uc_raw = tmin; has_u = 1; }\n        if (has_max) { lc_raw = tmax; has_l = 1; }\n      }\n      if (has_l && lower_counts"),
    ("divide_by_abs_coef", "  if (act_inf == 0) {\n    t = beta - act_fin;\n    t = t / a;",
     "  if (act_inf == 0) {\n    t = beta - act_fin;\n    t = t / fabs(a);"),
    ("lower_rounded_down", "    c = ceil(c - prm->eps_int);", "    c = floor(c - prm->eps_int);"),
    ("upper_rounded_up", "    c = floor(c + prm->eps_int);", "    c = ceil(c + prm->eps_int);"),
    ("in_round_visibility", "    row_activity(P, i, L, U, &A[0], &A[1], &minfin, &mininf, &maxfin, &maxinf);\n    for (int64_t k = P->row_ptr[i]; k < P->row_ptr[i + 1]; k++) {\n      double a = P->val[k];\n      if (a == 0.0) continue;\n      int32_t j = P->col[k];\n      int is_int = P->vartype[j] == 1;\n      double bmin = a > 0.0 ? L[j] : U[j];",
     "    row_activity(P, i, Ln, Un, &A[0], &A[1], &minfin, &mininf, &maxfin, &maxinf);\n    for (int64_t k = P->row_ptr[i]; k < P->row_ptr[i + 1]; k++) {\n      double a = P->val[k];\n      if (a == 0.0) continue;\n      int32_t j = P->col[k];\n      int is_int = P->vartype[j] == 1;\n      double bmin = a > 0.0 ? Ln[j] : Un[j];"),
    ("converged_round_off_by_one",
     "    if (!ch) {\n      *status = ORC_CONVERGED;\n      *rounds = r;",
     "    if (!ch) {\n      *status = ORC_CONVERGED;\n      *rounds = r - 1;"),
    ("one_inf_any_owner", "  } else if (act_inf == 1 && isinf(b)) {", "  } else if (act_inf == 1) {"),
    ("ties_away_from_zero", "  if (rbit && (sticky || (sig & 1u))) sig++;", "  if (rbit) sig++;"),
    ("infeasibility_ignored", "    if (inf) {\n      *status = ORC_INFEASIBLE;\n      *rounds = r;",
     "    if (0) {\n      *status = ORC_INFEASIBLE;\n      *rounds = r;"),
    ("no_continuous_threshold", "    sig = c > Lj + prm->cont_rel_tol * s;", "    sig = c > Lj;"),
    ("infinities_not_counted",
     "    if (isinf(bmin)) cmin++;\n    else acc_add_product(amin, a, bmin);",
     "    if (isinf(bmin)) cmin += 0;\n    else acc_add_product(amin, a, bmin);"),
    ("last_writer_wins", "        if (c > Ln[j]) Ln[j] = c;", "        Ln[j] = c;"),
    ("last_row_skipped", "  for (int32_t i = 0; i < P->m; i++) {\n    double minfin, maxfin;\n    int64_t mininf, maxinf;\n    row_activity(P, i, L, U,",
     "  for (int32_t i = 0; i < P->m - 1; i++) {\n    double minfin, maxfin;\n    int64_t mininf, maxinf;\n    row_activity(P, i, L, U,"),
    ("negative_products_added", "  int side = ((a < 0.0) != (b < 0.0)) ? 1 : 0;", "  int side = 0;"),
    ("store_rounds_nearest_not_down", "  if ((double)f > x) f = nextafterf(f, -INFINITY);",
     "  if (0) f = nextafterf(f, -INFINITY);"),
    ("store_rounds_inward", "static double store_up(double x) { return -store_down(-x) + 0.0; }",
     "static double store_up(double x) { return store_down(x); }"),
    ("store_keeps_subnormals", "  if (x > 0.0 && x < FLT_MIN) return 0.0;", "  if (0) return 0.0;"),
    ("store_not_applied_at_commit", "    if (prm->store32) {\n      Ln[j] = store_down(Ln[j]);",
     "    if (0) {\n      Ln[j] = store_down(Ln[j]);"),
    ("store_change_test_before_rounding",
     "    if (prm->store32) {\n      Ln[j] = store_down(Ln[j]);\n      Un[j] = store_up(Un[j]);\n    }\n    if (Ln[j] != L[j] || Un[j] != U[j]) ch = 1;",
     "    if (Ln[j] != L[j] || Un[j] != U[j]) ch = 1;\n    if (prm->store32) {\n      Ln[j] = store_down(Ln[j]);\n      Un[j] = store_up(Un[j]);\n    }"),
    ("store_input_not_rounded", "    if (prm->store32) {\n      lb[j] = store_down(lb[j]);",
     "    if (0) {\n      lb[j] = store_down(lb[j]);"),
    ("integer_input_not_rounded", "      lb[j] = ceil(lb[j] - prm->eps_int);\n      ub[j] = floor(ub[j] + prm->eps_int);",
     "      lb[j] = lb[j];\n      ub[j] = ub[j];"),
]

RUNNER = r"""
import sys, traceback
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import oracle, oracle_pins
orc = oracle.Oracle({lib!r})
failed = []
for chk in oracle_pins.ALL_CHECKS:
    try:
        chk(orc)
    except Exception as e:
        failed.append(chk.__name__)
print("FAILED_CHECKS", ",".join(failed))
sys.exit(0 if failed else 3)
"""


def test_mutant_table_matches_source():
    src = open(oracle.SOURCE).read()
    for name, old, new in MUTANTS:
        assert src.count(old) == 1, name


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new):
    src = open(oracle.SOURCE).read()
    assert src.count(old) == 1
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mutant.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        lib = oracle.compile_library(path, os.path.join(d, "libmutant.so"))
        code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
        try:
            p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                               timeout=240)
        except subprocess.TimeoutExpired:
            return  # a mutant that loops is caught as well
        assert p.returncode != 3, f"mutant {name} survived every pin:\n{p.stdout}\n{p.stderr}"
