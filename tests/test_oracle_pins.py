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


def _dense_h3(size, j, tau, nu1, nu2):
    """The size x size matrix I - tau v v^T, v = e_j + nu1 e_{j+1} + nu2 e_{j+2},
    written out (independent of the oracle's per-row loops)."""
    v = np.zeros(size)
    v[j], v[j + 1], v[j + 2] = 1.0, nu1, nu2
    return np.eye(size) - tau * np.outer(v, v)


@pytest.mark.parametrize("inverse", [False, True])
@pytest.mark.parametrize("left", [False, True])
def test_refl3_orders_brute_force(inverse, left):
    """Every order and side of the 3x3 oracle against the product of dense
    reflectors (any tau, nu1, nu2): right A H(0,0)...H(r-3,k-1), right
    inverse A H(r-3,k-1)...H(0,0), left H(r-3,k-1)...H(0,0) A, left inverse
    H(0,0)...H(r-3,k-1) A, r being the mixed dimension."""
    rng = np.random.default_rng(31 + 2 * inverse + left)
    m, n, k = 7, 6, 3
    r = m if left else n
    A0 = rng.standard_normal((m, n))
    TAU, NU1, NU2 = (rng.uniform(-1.5, 1.5, (r - 2, k)) for _ in range(3))
    order = [(j, p) for p in range(k) for j in range(r - 2)]  # Algorithm 2's order
    if inverse:
        order = order[::-1]
    ref = A0.copy()
    for j, p in order:
        H = _dense_h3(r, j, TAU[j, p], NU1[j, p], NU2[j, p])
        ref = H @ ref if left else ref @ H
    A = colmajor(A0, ld=m + 2)
    oracle.refl3seq(A, colmajor(TAU), colmajor(NU1), colmajor(NU2), inverse=inverse, left=left)
    assert np.allclose(np.asarray(A), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_refl3_inverse_undoes_forward():
    """With orthogonal reflectors (tau (1 + nu1^2 + nu2^2) = 2) the inverse
    call undoes the forward one, on both sides."""
    rng = np.random.default_rng(5)
    m, n, k = 9, 11, 4
    for left in (False, True):
        r = m if left else n
        NU1, NU2 = rng.standard_normal((r - 2, k)), rng.standard_normal((r - 2, k))
        TAU = 2.0 / (1.0 + NU1 ** 2 + NU2 ** 2)
        A0 = rng.standard_normal((m, n))
        A = colmajor(A0)
        T, N1, N2 = colmajor(TAU), colmajor(NU1), colmajor(NU2)
        oracle.refl3seq(A, T, N1, N2, left=left)
        assert not np.allclose(np.asarray(A), A0)
        oracle.refl3seq(A, T, N1, N2, left=left, inverse=True)
        assert np.allclose(np.asarray(A), A0, rtol=0, atol=1e-12)
