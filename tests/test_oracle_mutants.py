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
from oracle_pins import ALL_PINS

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
