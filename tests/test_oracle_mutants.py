"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of oracle.c (on the CPU, in a temporary
directory), builds it, and runs the pin suite against that build in a child
process: the suite has to fail.  All mutants keep every access in bounds.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "mv_sign": ("y[i] = y[i] + prod;", "y[i] = y[i] - prod;"),
    "mv_drop_last_term": ("for (int64_t p = ptr[j]; p < ptr[j + 1]; ++p) {\n            int64_t i = idx[p];",
                          "for (int64_t p = ptr[j]; p + 1 < ptr[j + 1]; ++p) {\n            int64_t i = idx[p];"),
    "vtm_wrong_vector_index": ("double prod = val[p] * v[idx[p]];\n            s = s + prod;",
                               "double prod = val[p] * v[idx[ptr[j]]];\n            s = s + prod;"),
    "csr_mv_uses_row_value": ("double prod = val[p] * x[idx[p]];\n            s = s + prod;",
                              "double prod = val[p] * x[idx[ptr[i]]];\n            s = s + prod;"),
    "csr_vtm_transposed": ("u[j] = u[j] + prod;", "u[j] = u[j] + val[p] * v[i % (j + 1)];"),
    "denominator_signed": ("if (d) d[i] = d[i] + fabs(val[p]) * fabs(x[j]);",
                           "if (d) d[i] = d[i] + val[p] * fabs(x[j]);"),
    "vtm_csc_denominator_inflated": ("a = a + fabs(val[p]) * fabs(v[idx[p]]);",
                                     "a = a + fabs(val[p]) * (fabs(v[idx[p]]) + 1.0);"),
    "csr_mv_denominator_inflated": ("a = a + fabs(val[p]) * fabs(x[idx[p]]);",
                                    "a = a + fabs(val[p]) * (fabs(x[idx[p]]) + 1.0);"),
    "csr_vtm_denominator_inflated": ("if (d) d[j] = d[j] + fabs(val[p]) * fabs(v[i]);",
                                     "if (d) d[j] = d[j] + fabs(val[p]) * (fabs(v[i]) + 1.0);"),
    "batch_denominator_is_output": ("if (D) scatter_col(D, out_len, ldd, c, dout);",
                                    "if (D) scatter_col(D, out_len, ldd, c, yout);"),
    "batch_denominator_wrong_column": ("if (D) scatter_col(D, out_len, ldd, c, dout);",
                                       "if (D) scatter_col(D, out_len, ldd, 0, dout);"),
    "round_one_bit_short": ("double q = ldexp(1.0, ex - (p - 1));", "double q = ldexp(1.0, ex - (p - 2));"),
    "round_truncates": ("double r = nearbyint(x / q) * q;", "double r = trunc(x / q) * q;"),
    "paper_offsets_off_by_one": ("(i < big ? q + 1 : q)", "(i + 1 < big ? q + 1 : q)"),
    "left_group_end_wrong": ("(needRight[i] == 0 || jf[i] != jl[i])", "(needRight[i] == 0 || jf[i] == jl[i])"),
    "backward_scan_folds_wrong_way": ("else seg_op(s, k, needRight[i], rightGroup[i], &s, &k);",
                                      "else seg_op(needRight[i], rightGroup[i], s, k, &s, &k);"),
    "seg_op_does_not_reset": ("else        { *rs = t;     *rk = l; }", "else        { *rs = s + t; *rk = l; }"),
    "zone_needs_three_groups": ("if (gfirst[j] >= 0 && glast[j] > gfirst[j]) {", "if (gfirst[j] >= 0 && glast[j] > gfirst[j] + 1) {"),
    "nzp_vtm_overwrites_zone": ("if (g > 0 && off[g] > ptr[j]) u[j] = u[j] + part;", "if (0) u[j] = u[j] + part;"),
    "nzp_mv_skips_first_group": ("for (int64_t r = 0; r < m; ++r) y[r] = y[r] + yi[r];",
                                 "for (int64_t r = 0; r < m; ++r) y[r] = g ? y[r] + yi[r] : y[r];"),
    "cover_last_is_first": ("jl[i] = col[off[i + 1] - 1];", "jl[i] = col[off[i]];"),
    "fixed_split_drops_short_chunk": ("int64_t G = (Z + C - 1) / C;", "int64_t G = Z / C;"),
    "colp_without_part_count": ("return (double)P * (double)(mx - mn) / (double)Z;",
                                "return (double)(mx - mn) / (double)Z;"),
    "colp_min_never_updated": ("if (mn < 0 || cnt < mn) mn = cnt;", "if (mn < 0) mn = cnt;"),
    "colp_long_spans_last": ("int64_t j1 = j0 + (i < big ? q + 1 : q);",
                             "int64_t j1 = j0 + (i >= P - big ? q + 1 : q);"),
    "cgls_residual_sign": ("r[i] = r[i] - alpha * q[i];", "r[i] = r[i] + alpha * q[i];"),
    "cgls_steepest_descent": ("const double beta = gamma > 0.0 ? gamma_new / gamma : 0.0;",
                              "const double beta = 0.0 * gamma_new;"),
    "cgls_step_from_direction_norm": ("const double delta = dot_seq(q, q, m);",
                                      "const double delta = dot_seq(p, p, n);"),
    "cgls_iterate_moves_along_gradient": ("x[j] = x[j] + alpha * p[j];", "x[j] = x[j] + alpha * s[j];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation site not found: " + name
    mutated = src.replace(old, new, 1)
    c_path = tmp_path / "oracle_mut.c"
    so_path = tmp_path / "liboracle_mut.so"
    c_path.write_text(mutated)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", str(so_path), str(c_path), "-lm"])
    env = dict(os.environ, SPW_ORACLE_LIB=str(so_path))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, "mutant %s survived the pins:\n%s" % (name, r.stdout[-2000:])
