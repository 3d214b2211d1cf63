"""The pins of the spec evaluator catch plausible mistakes in it.

Each case plants one mistake in a copy of oracle/spec_eval.py (a dropped
transpose, a dropped scale, a wrong sign, a reversed index in an outer
product, a dot of the wrong operands, a dropped update), loads the copy in place of the real module
and runs the evaluator's pin tests against it: at least one must fail.  The
real evaluator passes the same selection."""

import importlib.util

import pytest

from oracle import spec_eval
from tests import test_btoc_cpu as tb

SRC = open(spec_eval.__file__).read()

MUTANTS = {
    "transpose_ignored": ("M = a[1].T if a[3] else a[1]", "M = a[1]"),
    "scale_dropped": ('return ("vec", a[2] * r if a[2] != 1.0 else r)', 'return ("vec", r)'),
    "minus_is_plus": ('return ("vec", a[1] + sign * b[1] if sign < 0 else a[1] + b[1])',
                      'return ("vec", a[1] + b[1])'),
    "outer_reversed_index": ('return ("outer", np.outer(a[1], b[1]))',
                             'return ("outer", np.outer(a[1], b[1][::-1]))'),
    "dot_squares_first": ('return ("scal", float(np.dot(a[1], b[1])))',
                          'return ("scal", float(np.dot(a[1], a[1])))'),
    "scalar_times_vector_unscaled": ('return ("vec", s[1] * v[1])', 'return ("vec", v[1])'),
    "update_dropped": ('return ("mat", a[1] + b[1], 1.0, False)', 'return ("mat", a[1], 1.0, False)'),
}


def _checks():
    return [
        lambda: [tb.test_evaluator_hand_worked(k, o) for k, o in (
            ("bicgk", ("q", "s")), ("gemver", ("B", "x", "w")), ("atax", ("y",)),
            ("dgemvt", ("x", "w")), ("dgemv", ("z",)), ("gesummv", ("y",)),
            ("waxpby", ("w",)), ("vadd", ("x",)), ("axpydot", ("z", "r")))],
        lambda: tb.test_evaluator_agrees_with_the_oracle_kernels(7, 5),
        lambda: tb.test_evaluator_integers_exact(),
    ]


def _failures():
    bad = 0
    for check in _checks():
        try:
            check()
        except (AssertionError, ValueError, KeyError, IndexError):
            bad += 1
    return bad


def test_real_evaluator_passes_selection():
    assert _failures() == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    assert SRC.count(old) == 1, f"mutation site of {name} not unique"
    path = tmp_path / "spec_eval_mutant.py"
    path.write_text(SRC.replace(old, new))
    spec = importlib.util.spec_from_file_location("spec_eval_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    monkeypatch.setattr(tb.spec_eval, "evaluate", mod.evaluate)
    assert _failures() >= 1, f"no pin catches mutant {name}"
