"""The pins catch plausible mistakes in the oracle.

Each case plants one mistake (a dropped term, a wrong sign, a wrong index,
a transposed or swapped operand, an ignored leading dimension) in a copy of
the oracle's C source, builds it on the CPU, swaps it in for the real
library and runs a fixed selection of the pin tests against it: at least one
must fail.  The real oracle passes the same selection.
"""

import ctypes
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_exact as tx
from tests import test_oracle_properties as tp

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "bto_oracle.c")).read()

MUTANTS = {
    "rowdot_drops_last_term": ("for (int64_t j = 0; j < n; ++j)\n            acc += a[j] * v[j];",
                               "for (int64_t j = 0; j + 1 < n; ++j)\n            acc += a[j] * v[j];"),
    "rowdot_ignores_lda": ("const double *a = A + i * lda;\n        double acc",
                           "const double *a = A + i * n;\n        double acc"),
    "colsum_wrong_sign": ("out[j] += a[j] * vi;", "out[j] -= a[j] * vi;"),
    "colsum_drops_last_row": ("for (int64_t i = 0; i < m; ++i) {\n            const double *a = A + i * lda;\n            double vi",
                              "for (int64_t i = 0; i + 1 < m; ++i) {\n            const double *a = A + i * lda;\n            double vi"),
    "colsum_block_edge": ("for (int64_t j = j0; j < j1; ++j)\n                out[j] += a[j] * vi;",
                          "for (int64_t j = j0; j + 1 < j1; ++j)\n                out[j] += a[j] * vi;"),
    "gemver_u2_times_v1": ("b[j] = t + u2[i] * v2[j];", "b[j] = t + u2[i] * v1[j];"),
    "gemver_minus_z": ("    colsums(m, n, B, ldb, y, x);\n    for (int64_t j = 0; j < n; ++j)\n        x[j] = beta * x[j] + z[j];",
                       "    colsums(m, n, B, ldb, y, x);\n    for (int64_t j = 0; j < n; ++j)\n        x[j] = beta * x[j] - z[j];"),
    "gemver_w_from_A": ("rowdots(m, n, B, ldb, x, w);", "rowdots(m, n, A, lda, x, w);"),
    "gemver_scales_swapped": ("        x[j] = beta * x[j] + z[j];\n    rowdots(m, n, B",
                              "        x[j] = alpha * x[j] + z[j];\n    rowdots(m, n, B"),
    "atax_skips_Ax": ("    rowdots(m, n, A, lda, x, t);\n    colsums(m, n, A, lda, t, y);",
                      "    for (int64_t i = 0; i < m; ++i) t[i] = 1.0;\n    colsums(m, n, A, lda, t, y);"),
    "dgemvt_alpha_is_beta": ("        w[i] = alpha * w[i];\n}\n\n/* DGEMV",
                             "        w[i] = beta * w[i];\n}\n\n/* DGEMV"),
    "axpydot_plus": ("z[k] = w[k] - alpha * v[k];", "z[k] = w[k] + alpha * v[k];"),
    "pairwise_drops_element": ("pairwise_dot(x + h, y + h, len - h)", "pairwise_dot(x + h, y + h, len - h - 1)"),
    "pairwise_wrong_offset": ("pairwise_dot(x + h, y + h, len - h)", "pairwise_dot(x + h, y, len - h)"),
    "waxpby_beta_x": ("double b = beta * y[k];", "double b = beta * x[k];"),
    "vadd_adds_y_twice": ("x[k] = t + z[k];", "x[k] = t + y[k];"),
    "dgemv_drops_beta_y": ("        double b = beta * y[i];\n        z[i] = a + b;",
                           "        double b = beta * y[i];\n        z[i] = a + 0.0 * b;"),
    "dgemv_beta_times_dot": ("double b = beta * y[i];", "double b = beta * t[i];"),
    "gesummv_reads_A_twice": ("rowdots(m, n, B, ldb, x, t + m);", "rowdots(m, n, A, lda, x, t + m);"),
    "gesummv_ignores_ldb": ("rowdots(m, n, B, ldb, x, t + m);", "rowdots(m, n, B, lda, x, t + m);"),
    "gesummv_scales_swapped": ("double a = alpha * t[i];\n        double b = beta * t[m + i];",
                               "double a = beta * t[i];\n        double b = alpha * t[m + i];"),
}


def _checks():
    """The pin tests run against each mutant (each takes the oracle module)."""
    return [
        lambda o: tx.test_bicgk_rational(o, 3, 5),
        lambda o: tx.test_gemver_rational(o, 3, 8),
        lambda o: tx.test_atax_rational(o, 5, 3),
        lambda o: tx.test_dgemvt_rational(o, 3, 8),
        lambda o: tx.test_dgemv_gesummv_rational(o, 3, 8),
        lambda o: tx.test_axpydot_rational(o, 300),
        lambda o: tx.test_waxpby_vadd_rational(o, 5),
        lambda o: tx.test_golden_hand_worked(o),
        lambda o: tx.test_integer_exact_matrix_kernels(o, 300, 257),
        lambda o: tx.test_integer_exact_vector_kernels(o, 4097),
        lambda o: tp.test_identity(o, 300),
        lambda o: tp.test_bicgk_invariant(o, 200, 150),
        lambda o: tp.test_lda_padding_is_ignored(o, 130, 257, 300),
    ]


def _failures(mod):
    bad = 0
    for check in _checks():
        try:
            check(mod)
        except AssertionError:
            bad += 1
    return bad


def test_real_oracle_passes_selection():
    assert _failures(oracle) == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    assert SRC.count(old) == 1, f"mutation site of {name} not unique"
    src = tmp_path / "mutant.c"
    src.write_text(SRC.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", *oracle.CFLAGS, "-o", str(lib), str(src)], check=True)
    monkeypatch.setattr(oracle, "_lib", oracle.bind(ctypes.CDLL(str(lib))))
    assert _failures(oracle) >= 1, f"no pin catches mutant {name}"
