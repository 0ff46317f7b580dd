"""The CPU oracle against its pins (brute force, exact arithmetic, BLAS,
closed forms, invariants, a hand-worked example).  CPU only."""
import numpy as np
import pytest

import oracle
from oracle_pins import (ALL_PINS, LEFT_PINS, REFL3_PINS, REFL_PINS, colmajor, pin_left_is_right_on_transpose,
                         pin_refl3_closed_forms, rand_problem)


def oracle_apply(A, C, S, inverse=False):
    oracle.rotseq(A, C, S, inverse=inverse)


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin(oracle_apply)


def test_threaded_driver_bitwise():
    """Row-partitioned threads give the single-thread result bitwise."""
    rng = np.random.Generator(np.random.PCG64(7))
    A, C, S = rand_problem(rng, 101, 40, 9, lda=103)
    ref = np.array(A)
    oracle.rotseq(colmajor(ref), C, S)
    one = colmajor(np.array(A), 103)
    oracle.rotseq(one, C, S)
    for t in (2, 3, 8, 200):
        B = colmajor(np.array(A), 103)
        oracle.rotseq(B, C, S, threads=t)
        assert np.array_equal(np.asarray(B), np.asarray(one))


def test_quick_returns():
    """m = 0, n <= 1 or k = 0 leave A untouched."""
    rng = np.random.Generator(np.random.PCG64(8))
    A = colmajor(rng.standard_normal((4, 1)))
    before = np.array(A)
    oracle.rotseq(A, colmajor(np.zeros((0, 3))), colmajor(np.zeros((0, 3))))
    assert np.array_equal(np.asarray(A), before)
    A, C, S = rand_problem(rng, 4, 5, 0)
    before = np.array(A)
    oracle.rotseq(A, C, S)
    assert np.array_equal(np.asarray(A), before)


def oracle_left(A, C, S, inverse=False):
    oracle.rotseq(A, C, S, inverse=inverse, left=True)


def oracle_refl(A, TAU, NU, inverse=False, left=False):
    oracle.reflseq(A, TAU, NU, inverse=inverse, left=left)


@pytest.mark.parametrize("pin", LEFT_PINS, ids=lambda p: p.__name__)
def test_left_pin(pin):
    pin(oracle_left)


def test_left_is_right_on_transpose():
    pin_left_is_right_on_transpose(oracle_left, oracle_apply)


@pytest.mark.parametrize("pin", REFL_PINS, ids=lambda p: p.__name__)
def test_refl_pin(pin):
    pin(oracle_refl)


def oracle_refl3(A, TAU, NU1, NU2):
    oracle.refl3seq(A, TAU, NU1, NU2)


@pytest.mark.parametrize("pin", REFL3_PINS, ids=lambda p: p.__name__)
def test_refl3_pin(pin):
    pin(oracle_refl3)


def test_refl3_closed_forms():
    pin_refl3_closed_forms(oracle_refl3, oracle_refl)


def test_refl3_quick_returns():
    """n <= 2 and k = 0 leave A alone; mismatched coefficient shapes raise."""
    A = colmajor(np.arange(6.0).reshape(3, 2))
    oracle.refl3seq(A, colmajor(np.zeros((0, 2))), colmajor(np.zeros((0, 2))), colmajor(np.zeros((0, 2))))
    assert np.array_equal(np.asarray(A), np.arange(6.0).reshape(3, 2))
    with pytest.raises(ValueError):
        oracle.refl3seq(colmajor(np.zeros((2, 5))), colmajor(np.zeros((3, 1))), colmajor(np.zeros((3, 2))),
                        colmajor(np.zeros((3, 1))))
