"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each mutant is one plausible slip (a dropped term, a wrong sign or index, a
transposed operand, a missing check) made by a text substitution on a copy of
``oracle/cg_oracle.c``; the copy is compiled to a temporary library and the
whole pin set of ``tests/pins.py`` is run against it in a child process
(a mutant may crash: that counts as caught).  The real oracle is never
modified.
"""
import concurrent.futures as cf
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "cg_oracle.c")

MUTANTS = {
    "csr_drops_last_term": ("k < ptr[i + 1]; ++k)\n            s += val[k] * x[col[k]];",
                            "k + 1 < ptr[i + 1]; ++k)\n            s += val[k] * x[col[k]];"),
    "csr_wrong_x_index": ("s += val[k] * x[col[k]];", "s += val[k] * x[i];"),
    "csc_transposed_operand": ("y[row[k]] += val[k] * x[j];", "y[j] += val[k] * x[row[k]];"),
    "sym_missing_mirror": ("            if (j != i)\n                y[j] += val[k] * x[i];\n", ""),
    "sym_mirror_wrong_x": ("y[j] += val[k] * x[i];", "y[j] += val[k] * x[j];"),
    "sym_diagonal_twice": ("if (j != i)\n                y[j]", "if (j >= i)\n                y[j]"),
    "dot_drops_first_term": ("for (int64_t i = 0; i < n; ++i) {\n        const double p = a[i] * b[i];",
                             "for (int64_t i = 1; i < n; ++i) {\n        const double p = a[i] * b[i];"),
    "dot_drops_product_error": ("c += e + pe;", "c += e;"),
    "dot_drops_sum_error": ("c += e + pe;", "c += pe;"),
    "dot_plain_drops_last_term": ("for (int64_t i = 0; i < n; ++i)\n        s += a[i] * b[i];",
                                  "for (int64_t i = 0; i + 1 < n; ++i)\n        s += a[i] * b[i];"),
    "dot_pairwise_drops_term": ("return orc_dot_pairwise(h, a, b) + orc_dot_pairwise(n - h, a + h, b + h);",
                                "return orc_dot_pairwise(h, a, b) + orc_dot_pairwise(n - h - 1, a + h, b + h);"),
    "dot_pairwise_leaf_skips_first": ("for (int64_t i = 0; i < n; ++i)\n            s += a[i] * b[i];\n        return s;",
                                      "for (int64_t i = 1; i < n; ++i)\n            s += a[i] * b[i];\n        return s;"),
    "dot_fused_drops_first": ("for (int64_t i = 0; i < n; ++i)\n        s = fma(a[i], b[i], s);",
                              "for (int64_t i = 1; i < n; ++i)\n        s = fma(a[i], b[i], s);"),
    "cg_fused_x_update_sign": ("x[i] = fma(alpha, p[i], x[i]);", "x[i] = fma(-alpha, p[i], x[i]);"),
    "cg_fused_r_update_sign": ("r[i] = fma(-alpha, q[i], r[i]);", "r[i] = fma(alpha, q[i], r[i]);"),
    "cg_fused_p_update_operand": ("p[i] = fma(beta, p[i], r[i]);", "p[i] = fma(beta, r[i], r[i]);"),
    "cg_fused_mode_ignored": ("const int fused = dot_mode == 3;", "const int fused = 0;"),
    "cg_snapshot_index_off": ("memcpy(x_hist + (size_t)((k - x_first) / x_stride) * (size_t)n",
                              "memcpy(x_hist + (size_t)((k - x_first) / x_stride + 1 == x_cap ? 0 : (k - x_first) / x_stride + 1) * (size_t)n"),
    "cg_x_update_sign": ("x[i] = x[i] + alpha * p[i];", "x[i] = x[i] - alpha * p[i];"),
    "cg_r_update_sign": ("r[i] = r[i] - alpha * q[i];", "r[i] = r[i] + alpha * q[i];"),
    "cg_beta_inverted": ("double beta = rho_new / rho;", "double beta = rho / rho_new;"),
    "cg_p_update_operand": ("p[i] = r[i] + beta * p[i];", "p[i] = r[i] + beta * r[i];"),
    "cg_init_residual_sign": ("r[i] = b[i] - q[i];\n        p[i] = r[i];", "r[i] = b[i] + q[i];\n        p[i] = r[i];"),
    "cg_absolute_criterion": ("            if (sqrt(rho) <= tol * nb) {\n                status = ORC_OK;\n                break;",
                              "            if (sqrt(rho) <= tol) {\n                status = ORC_OK;\n                break;"),
    "cg_alpha_inverted": ("double alpha = rho / sigma;", "double alpha = sigma / rho;"),
    "cg_no_breakdown_check": ("if (!(sigma > 0.0) || !isfinite(sigma)) {", "if (!isfinite(sigma)) {"),
    "cg_no_nonfinite_check": ("if (!isfinite(nb)) {", "if (0) {"),
    "cg_iters_off_by_one": ("info->iters = k;", "info->iters = k + 1;"),
    "cg_true_residual_unscaled": ("info->relres_true = sqrt(dot(n, r, r)) / nb;",
                                  "info->relres_true = sqrt(dot(n, r, r));"),
    "transpose_wrong_index": ("tidx[dst] = (int32_t)l;", "tidx[dst] = idx[k];"),
    "upper_drops_diagonal": ("if (col[k] >= i) {", "if (col[k] > i) {"),
    "expand_drops_lower": ("if (tidx[k] < i) {", "if (tidx[k] < 0) {"),
    "validate_misses_duplicates": ("if (k > b && idx[k] <= idx[k - 1])", "if (k > b && idx[k] < idx[k - 1])"),
    "validate_misses_diagonal_first": ("k == b && j != l)", "k == b && j < l)"),
    "validate_accepts_empty_sym_row": ("if (fmt == ORC_FMT_SYM_CSR && e == b)", "if (fmt == ORC_FMT_SYM_CSR && e < b)"),
}


TIMING_MODE_MARK = "/* ------------------------------------------------------- timing mode */"


def _run_mutant(name, tmpdir):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    # mistakes are planted in the reference functions only, not in the OpenMP
    # timing mode at the end of the file (which repeats some of their lines)
    cut = src.index(TIMING_MODE_MARK)
    ref, timing = src[:cut], src[cut:]
    assert ref.count(old) == 1, f"mutation site for {name} not unique"
    msrc = os.path.join(tmpdir, f"{name}.c")
    mlib = os.path.join(tmpdir, f"{name}.so")
    with open(msrc, "w") as f:
        f.write(ref.replace(old, new) + timing)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-D_POSIX_C_SOURCE=199309L", "-fopenmp", "-fPIC",
                    "-shared", "-o", mlib, msrc, "-lm"], check=True)
    p = subprocess.run([sys.executable, "-m", "tests.pins", mlib], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    if p.returncode != 0:
        return name, [f"child exited {p.returncode}"]
    return name, json.loads(p.stdout.strip().splitlines()[-1])


def test_every_planted_mistake_is_caught(tmp_path):
    with cf.ThreadPoolExecutor(max_workers=6) as ex:
        results = dict(ex.map(lambda nm: _run_mutant(nm, str(tmp_path)), MUTANTS))
    survivors = [nm for nm, failed in results.items() if not failed]
    assert not survivors, f"mutants not caught by any pin: {survivors}"


def test_real_oracle_passes_all_pins():
    from tests import pins
    import oracle
    assert pins.run_all(oracle.build.LIB if os.path.exists(oracle.build.LIB) else oracle.build.build()) == []


if __name__ == "__main__":
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        for nm in MUTANTS:
            print(_run_mutant(nm, d))
    pytest.main([__file__])
