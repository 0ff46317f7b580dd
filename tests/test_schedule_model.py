"""The GPU sweep's schedule, replayed on the CPU, against the oracle."""
import numpy as np
import pytest

import oracle
from oracle_pins import colmajor, rand_problem
from schedule_model import sweep

SHAPES = [(5, 2, 1), (7, 3, 5), (9, 17, 3), (4, 30, 16), (6, 12, 40), (3, 40, 33), (2, 5, 9)]


@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("band", [0, 1, 2, 4, 8, 16])
def test_exact_schedule_is_bitwise_algorithm2(m, n, k, band):
    rng = np.random.Generator(np.random.PCG64(m * 1000 + n * 10 + k))
    A, C, S = rand_problem(rng, m, n, k)
    ref = colmajor(np.array(A))
    oracle.rotseq(ref, C, S)
    got = sweep(np.array(A), np.asarray(C), np.asarray(S), band=band, arith="exact")
    assert np.array_equal(got, np.asarray(ref))


@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("band", [0, 1, 4, 16])
def test_lifting_sign_bookkeeping(m, n, k, band):
    """Lifting coefficients with column signs give Algorithm 2's result."""
    rng = np.random.Generator(np.random.PCG64(m * 7 + n * 3 + k))
    A, C, S = rand_problem(rng, m, n, k)
    ref = colmajor(np.array(A))
    oracle.rotseq(ref, C, S)
    got = sweep(np.array(A), np.asarray(C), np.asarray(S), band=band, arith="lift")
    err = np.linalg.norm(got - np.asarray(ref)) / np.linalg.norm(np.asarray(A))
    assert err < 1e-13


def test_lifting_all_negative_cosines():
    """Every rotation with c < 0 flips signs; the bookkeeping must undo them."""
    rng = np.random.Generator(np.random.PCG64(11))
    m, n, k = 4, 9, 7
    A = colmajor(rng.standard_normal((m, n)))
    th = rng.uniform(0.6 * np.pi, 1.4 * np.pi, (n - 1, k))
    C, S = colmajor(np.cos(th)), colmajor(np.sin(th))
    ref = colmajor(np.array(A))
    oracle.rotseq(ref, C, S)
    got = sweep(np.array(A), np.asarray(C), np.asarray(S), band=4, arith="lift")
    assert np.linalg.norm(got - np.asarray(ref)) / np.linalg.norm(np.asarray(A)) < 1e-13


@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("band", [1, 4, 8])
def test_reflector_sign_bookkeeping(m, n, k, band):
    """Reflectors as rotations plus tracked right-column negations (the
    device's prep for rotseq_refl_ex_*) give the oracle's reflector loop; the
    column-reversed reading gives its reverse loop."""
    from paper_2412_01852_amd.inputs import make_reflectors
    rng = np.random.Generator(np.random.PCG64(m * 5 + n * 11 + k))
    A0 = rng.standard_normal((m, n))
    tau, nu = make_reflectors(n - 1, k, rng, identity_frac=0.2)
    tau, nu = np.array(tau), np.array(nu)
    ref = colmajor(A0)
    oracle.reflseq(ref, colmajor(tau), colmajor(nu))
    got = sweep(A0.copy(), tau, nu, band=band, arith="lift", kind="reflect")
    assert np.linalg.norm(got - np.asarray(ref)) / np.linalg.norm(A0) < 1e-13
    # reverse order: the forward sweep on A[:, ::-1] with C/S read backwards
    ref = colmajor(A0)
    oracle.reflseq(ref, colmajor(tau), colmajor(nu), inverse=True)
    got = sweep(A0[:, ::-1].copy(), tau[::-1, ::-1].copy(), nu[::-1, ::-1].copy(), band=band,
                arith="lift", kind="reflect_rev")[:, ::-1]
    assert np.linalg.norm(got - np.asarray(ref)) / np.linalg.norm(A0) < 1e-13
