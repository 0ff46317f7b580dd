"""Strength of the oracle pins: broken copies of the oracle must fail.

Each mutant is the oracle source with one plausible mistake planted (a sign,
a dropped term, a transposed operand, a wrong loop order or bound, a wrong
leading dimension), compiled on the CPU into a temporary library.  The pins
of oracle_pins.py must reject every one of them.
"""
import os

import pytest

import oracle
from oracle import build as obuild
from oracle_pins import (ALL_PINS, LEFT_PINS, REFL3_PINS, REFL_PINS, pin_left_is_right_on_transpose,
                         pin_refl3_closed_forms)

FWD_LOOP = ("    for (int64_t p = 0; p < k; ++p)\n"
            "        for (int64_t j = 0; j + 1 < n; ++j)\n"
            "            rot(m, &A[j * lda], &A[(j + 1) * lda], C[j + p * ldc], S[j + p * lds]);")

MUTANTS = {
    "y_sign": ("y[i] = -s * x[i] + c * y[i];", "y[i] = s * x[i] + c * y[i];"),
    "x_sign": ("double t = c * x[i] + s * y[i];", "double t = c * x[i] - s * y[i];"),
    "dropped_term": ("double t = c * x[i] + s * y[i];", "double t = c * x[i];"),
    "x_not_written": ("x[i] = t;", "(void)t;"),
    "y_uses_new_x": ("        y[i] = -s * x[i] + c * y[i];\n        x[i] = t;",
                     "        x[i] = t;\n        y[i] = -s * x[i] + c * y[i];"),
    "j_descending": (FWD_LOOP, FWD_LOOP.replace("for (int64_t j = 0; j + 1 < n; ++j)",
                                                "for (int64_t j = n - 2; j >= 0; --j)")),
    "loops_swapped": (FWD_LOOP, FWD_LOOP.replace(
        "for (int64_t p = 0; p < k; ++p)\n        for (int64_t j = 0; j + 1 < n; ++j)",
        "for (int64_t j = 0; j + 1 < n; ++j)\n        for (int64_t p = 0; p < k; ++p)")),
    "c_transposed_index": (FWD_LOOP, FWD_LOOP.replace("C[j + p * ldc]", "C[p + j * ldc]")),
    "cs_swapped": (FWD_LOOP, FWD_LOOP.replace("C[j + p * ldc], S[j + p * lds]",
                                              "S[j + p * lds], C[j + p * ldc]")),
    "wrong_ld_for_c": (FWD_LOOP, FWD_LOOP.replace("C[j + p * ldc]", "C[j + p * lds]")),
    "last_pair_skipped": (FWD_LOOP, FWD_LOOP.replace("j + 1 < n", "j + 2 < n")),
    "last_sequence_skipped": (FWD_LOOP, FWD_LOOP.replace("p < k", "p + 1 < k")),
    "inverse_not_transposed": ("C[j + p * ldc], -S[j + p * lds]", "C[j + p * ldc], S[j + p * lds]"),
    "inverse_forward_order": ("    for (int64_t p = k - 1; p >= 0; --p)\n"
                              "        for (int64_t j = n - 2; j >= 0; --j)",
                              "    for (int64_t p = 0; p < k; ++p)\n"
                              "        for (int64_t j = 0; j + 1 < n; ++j)"),
}


LEFT_LOOP = ("        for (int64_t j = 0; j + 1 < m; ++j)\n"
             "            rot_rows(n, &A[j], &A[j + 1], lda, C[j + p * ldc], S[j + p * lds]);")

# Mutants of the left-application functions, caught by the left pins.
LEFT_MUTANTS = {
    "left_y_sign": ("y[i * ld] = -s * x[i * ld] + c * y[i * ld];",
                    "y[i * ld] = s * x[i * ld] + c * y[i * ld];"),
    "left_unit_stride": ("double t = c * x[i * ld] + s * y[i * ld];\n        y[i * ld] = -s * x[i * ld] + c * y[i * ld];\n        x[i * ld] = t;",
                         "double t = c * x[i] + s * y[i];\n        y[i] = -s * x[i] + c * y[i];\n        x[i] = t;"),
    "left_bound_uses_n": (LEFT_LOOP, LEFT_LOOP.replace("j + 1 < m", "j + 1 < n")),
    "left_row_roles_swapped": (LEFT_LOOP, LEFT_LOOP.replace("rot_rows(n, &A[j], &A[j + 1], lda",
                                                            "rot_rows(n, &A[j + 1], &A[j], lda")),
    "left_inverse_not_transposed": ("rot_rows(n, &A[j], &A[j + 1], lda, C[j + p * ldc], -S[j + p * lds]);",
                                    "rot_rows(n, &A[j], &A[j + 1], lda, C[j + p * ldc], S[j + p * lds]);"),
}

REFL_FWD = ("refl(m, &A[j * lda], &A[(j + 1) * lda], 1, TAU[j + p * ldt], NU[j + p * ldn]);")

# Mutants of the reflector functions, caught by the reflector pins.
REFL_MUTANTS = {
    "refl_w_roles_swapped": ("double w = x[i * stride] + nu * y[i * stride];",
                             "double w = nu * x[i * stride] + y[i * stride];"),
    "refl_x_sign": ("x[i * stride] = x[i * stride] - tau * w;", "x[i * stride] = x[i * stride] + tau * w;"),
    "refl_y_drops_nu": ("double tn = tau * nu;", "double tn = tau;"),
    "refl_y_uses_nu_squared": ("double tn = tau * nu;", "double tn = tau * nu * nu;"),
    "refl_w_uses_new_x": ("        double w = x[i * stride] + nu * y[i * stride];\n        x[i * stride] = x[i * stride] - tau * w;\n        y[i * stride] = y[i * stride] - tn * w;",
                          "        double w = x[i * stride] + nu * y[i * stride];\n        x[i * stride] = x[i * stride] - tau * w;\n        y[i * stride] = y[i * stride] - tn * (x[i * stride] + nu * y[i * stride]);"),
    "refl_tau_nu_swapped": (REFL_FWD, REFL_FWD.replace("TAU[j + p * ldt], NU[j + p * ldn]", "NU[j + p * ldn], TAU[j + p * ldt]")),
    "refl_inverse_forward_order": ("    for (int64_t p = k - 1; p >= 0; --p)\n"
                                   "        for (int64_t j = n - 2; j >= 0; --j)\n"
                                   "            refl(",
                                   "    for (int64_t p = 0; p < k; ++p)\n"
                                   "        for (int64_t j = 0; j + 1 < n; ++j)\n"
                                   "            refl("),
    "refl_left_wrong_stride": ("refl(n, &A[j], &A[j + 1], lda,", "refl(n, &A[j], &A[j + 1], 1,"),
}


# Mutants of the 3x3 reflector sequence, caught by the 3x3 reflector pins.
REFL3_LOAD = "double tau = TAU[j + p * ldt], nu1 = NU1[j + p * ld1], nu2 = NU2[j + p * ld2];"
REFL3_MUTANTS = {
    "refl3_w_drops_nu2": ("double w = x[i] + nu1 * y[i] + nu2 * z[i];", "double w = x[i] + nu1 * y[i];"),
    "refl3_z_uses_t1": ("z[i] = z[i] - t2 * w;", "z[i] = z[i] - t1 * w;"),
    "refl3_x_sign": ("x[i] = x[i] - tau * w;", "x[i] = x[i] + tau * w;"),
    "refl3_t2_uses_nu1": ("double t1 = tau * nu1, t2 = tau * nu2;", "double t1 = tau * nu1, t2 = tau * nu1;"),
    "refl3_nu_swapped": (REFL3_LOAD, "double tau = TAU[j + p * ldt], nu1 = NU2[j + p * ld2], nu2 = NU1[j + p * ld1];"),
    "refl3_window_overlaps": ("*z = &A[(j + 2) * lda];", "*z = &A[(j + 1) * lda];"),
    "refl3_last_reflector_dropped": ("for (int64_t j = 0; j + 2 < n; ++j) {", "for (int64_t j = 0; j + 3 < n; ++j) {"),
    "refl3_loops_swapped": ("    for (int64_t p = 0; p < k; ++p)\n        for (int64_t j = 0; j + 2 < n; ++j) {",
                            "    for (int64_t j = 0; j + 2 < n; ++j)\n        for (int64_t p = 0; p < k; ++p) {"),
}


@pytest.fixture(scope="module")
def source():
    with open(os.path.join(os.path.dirname(oracle.__file__), "rotseq_oracle.c")) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, source, tmp_path):
    old, new = MUTANTS[name]
    assert source.count(old) >= 1, f"mutation site for {name} not found"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new, 1))
    lib = oracle._load(obuild.build(str(src), str(tmp_path / "libmutant.so"),
                                    extra=["-Wno-unused-variable", "-Wno-unused-but-set-variable"]))

    def apply(A, C, S, inverse=False):
        oracle.rotseq(A, C, S, inverse=inverse, lib=lib)

    failed = []
    for pin in ALL_PINS:
        try:
            pin(apply)
        except AssertionError as e:
            failed.append((pin.__name__, str(e)[:80]))
    assert failed, f"mutant {name} passed every pin"


def _mutant_lib(source, tmp_path, old, new, name):
    assert source.count(old) >= 1, f"mutation site for {name} not found"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new, 1))
    return oracle._load(obuild.build(str(src), str(tmp_path / "libmutant.so"),
                                     extra=["-Wno-unused-variable", "-Wno-unused-but-set-variable",
                                            "-Wno-unused-parameter"]))


def _fails_some(pins, *fns):
    failed = []
    for pin in pins:
        try:
            pin(*fns)
        except AssertionError as e:
            failed.append((pin.__name__, str(e)[:80]))
    return failed


@pytest.mark.parametrize("name", sorted(LEFT_MUTANTS))
def test_left_mutant_is_caught(name, source, tmp_path):
    lib = _mutant_lib(source, tmp_path, *LEFT_MUTANTS[name], name)

    def left(A, C, S, inverse=False):
        oracle.rotseq(A, C, S, inverse=inverse, left=True, lib=lib)

    def right(A, C, S, inverse=False):
        oracle.rotseq(A, C, S, inverse=inverse, lib=lib)

    failed = _fails_some(LEFT_PINS, left)
    try:
        pin_left_is_right_on_transpose(left, right)
    except AssertionError as e:
        failed.append(("pin_left_is_right_on_transpose", str(e)[:80]))
    assert failed, f"mutant {name} passed every left pin"


@pytest.mark.parametrize("name", sorted(REFL_MUTANTS))
def test_refl_mutant_is_caught(name, source, tmp_path):
    lib = _mutant_lib(source, tmp_path, *REFL_MUTANTS[name], name)

    def refl(A, TAU, NU, inverse=False, left=False):
        oracle.reflseq(A, TAU, NU, inverse=inverse, left=left, lib=lib)

    assert _fails_some(REFL_PINS, refl), f"mutant {name} passed every reflector pin"


@pytest.mark.parametrize("name", sorted(REFL3_MUTANTS))
def test_refl3_mutant_is_caught(name, source, tmp_path):
    lib = _mutant_lib(source, tmp_path, *REFL3_MUTANTS[name], name)

    def refl3(A, TAU, NU1, NU2):
        oracle.refl3seq(A, TAU, NU1, NU2, lib=lib)

    def refl2(A, TAU, NU):
        oracle.reflseq(A, TAU, NU, lib=lib)

    failed = _fails_some(REFL3_PINS, refl3)
    try:
        pin_refl3_closed_forms(refl3, refl2)
    except AssertionError as e:
        failed.append(("pin_refl3_closed_forms", str(e)[:80]))
    assert failed, f"mutant {name} passed every 3x3 reflector pin"
