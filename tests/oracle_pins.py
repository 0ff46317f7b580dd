"""Pins that tie the CPU oracle to facts fixed outside of it.

Each pin takes ``apply(A, C, S, inverse=False)`` (an in-place rotation
sequence on column-major float64 views) and raises AssertionError when the
implementation disagrees with

* brute force: the dense n x n product of the rotation matrices G(j, p)
  (Algorithms 1 and 2 define A <- A G(0,0) ... G(n-2,k-1); G(j,p) is the
  identity except G[j][j] = G[j+1][j+1] = c, G[j+1][j] = s, G[j][j+1] = -s),
* exact rational arithmetic on the same floating-point inputs,
* the reference BLAS routine drot (one sequence, k = 1),
* closed forms (swap rotations, identity, reflection by -1, n = 2
  composition) and the invariants of orthogonal transforms,
* a hand-worked example stored under tests/golden/.

The same pins are run against deliberately broken copies of the oracle
(tests/test_oracle_mutants.py) to show that each plausible mistake is caught.
"""
from fractions import Fraction
import math
import os

import numpy as np

U = 2.0 ** -53  # unit roundoff of IEEE binary64
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def colmajor(arr, ld=None, fill=-999.5):
    arr = np.asarray(arr, dtype=np.float64)
    rows, cols = arr.shape
    ld = max(1, rows) if ld is None else ld
    buf = np.full((ld, max(cols, 1)), fill, dtype=np.float64, order="F")
    buf[:rows, :cols] = arr
    return buf[:rows, :cols]


def rand_problem(rng, m, n, k, lda=None, ldc=None, lds=None):
    A = colmajor(rng.standard_normal((m, n)), lda)
    th = rng.uniform(0, 2 * math.pi, (max(n - 1, 0), k))
    return A, colmajor(np.cos(th), ldc), colmajor(np.sin(th), lds)


def dense_q(C, S, n):
    """Q = prod_p prod_j G(j, p) in Algorithm 2's order, as a dense matrix."""
    Q = np.eye(n)
    nm1, k = C.shape
    for p in range(k):
        for j in range(nm1):
            G = np.eye(n)
            c, s = C[j, p], S[j, p]
            G[j, j] = c
            G[j + 1, j + 1] = c
            G[j + 1, j] = s
            G[j, j + 1] = -s
            Q = Q @ G
    return Q


def relerr(X, Y):
    den = np.linalg.norm(Y)
    return np.linalg.norm(X - Y) / (den if den else 1.0)


def _padding(A):
    buf = A.base if A.base is not None else A
    return buf[A.shape[0]:, :].copy()


# ---------------------------------------------------------------- pins

def pin_dense_bruteforce(apply):
    """P-1: A G(0,0)...G(n-2,k-1) computed densely; also lda/ldc/lds padding."""
    rng = np.random.Generator(np.random.PCG64(101))
    cases = [(1, 2, 1), (3, 2, 4), (5, 3, 1), (4, 5, 3), (7, 8, 5), (8, 12, 4),
             (6, 9, 9)]
    for idx, (m, n, k) in enumerate(cases):
        lda = m + (idx % 3)
        ldc = n - 1 + (idx % 2)
        lds = n - 1 + 2 * (idx % 2)
        A, C, S = rand_problem(rng, m, n, k, lda, ldc, lds)
        ref = np.asarray(A) @ dense_q(np.asarray(C), np.asarray(S), n)
        pad = _padding(A)
        apply(A, C, S)
        e = relerr(A, ref)
        assert e <= 1e-14, f"dense brute force m={m} n={n} k={k}: rel err {e:.3e}"
        assert np.array_equal(_padding(A), pad), "padding rows of A were modified"


def pin_inverse_dense(apply):
    """The inverse applies Q^T: A Q^T computed densely."""
    rng = np.random.Generator(np.random.PCG64(102))
    for (m, n, k) in [(3, 4, 2), (5, 7, 3), (2, 2, 5)]:
        A, C, S = rand_problem(rng, m, n, k, lda=m + 1)
        ref = np.asarray(A) @ dense_q(np.asarray(C), np.asarray(S), n).T
        apply(A, C, S, inverse=True)
        e = relerr(A, ref)
        assert e <= 1e-14, f"inverse vs dense m={m} n={n} k={k}: rel err {e:.3e}"


def _frac_matmul(X, Y):
    rows, inner, cols = len(X), len(Y), len(Y[0])
    return [[sum((X[i][t] * Y[t][j] for t in range(inner)), Fraction(0))
             for j in range(cols)] for i in range(rows)]


def pin_exact_rational(apply):
    """P-2: exact result of the same float inputs, via rational dense product.

    Rounding bound used: every entry of a row takes part in at most 2k of the
    (n-1)k rotations, each rotation commits at most 3u relative error per
    output entry (two products and one sum), and orthogonal propagation does
    not grow earlier errors, so ||row error|| <= 6 u (n-1) k ||row||.
    """
    # Pythagorean triples give well-conditioned rotations close to rationals.
    triples = [(3, 4, 5), (5, 12, 13), (8, 15, 17), (7, 24, 25), (20, 21, 29)]
    rng = np.random.Generator(np.random.PCG64(103))
    m, n, k = 3, 6, 4
    C = np.empty((n - 1, k))
    S = np.empty((n - 1, k))
    for p in range(k):
        for j in range(n - 1):
            a, b, h = triples[(j + 2 * p) % len(triples)]
            sg = -1.0 if (j + p) % 3 == 0 else 1.0
            C[j, p] = sg * a / h
            S[j, p] = b / h if p % 2 == 0 else -b / h
    A0 = rng.integers(-9, 10, (m, n)).astype(np.float64)
    Qf = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for p in range(k):
        for j in range(n - 1):
            G = [[Fraction(int(r == s)) for s in range(n)] for r in range(n)]
            c, s = Fraction(C[j, p]), Fraction(S[j, p])
            G[j][j] = c
            G[j + 1][j + 1] = c
            G[j + 1][j] = s
            G[j][j + 1] = -s
            Qf = _frac_matmul(Qf, G)
    Af = [[Fraction(float(v)) for v in row] for row in A0]
    exact = _frac_matmul(Af, Qf)
    A = colmajor(A0)
    apply(A, colmajor(C), colmajor(S))
    for i in range(m):
        err = math.sqrt(sum(float(Fraction(A[i, j]) - exact[i][j]) ** 2 for j in range(n)))
        nrm = float(np.linalg.norm(A0[i]))
        bound = 6 * U * (n - 1) * k * nrm
        assert err <= bound, f"row {i}: error {err:.3e} above bound {bound:.3e}"


def pin_drot(apply):
    """P-3: one sequence equals the BLAS drot routine applied for j = 0..n-2."""
    from scipy.linalg import blas
    rng = np.random.Generator(np.random.PCG64(104))
    m, n = 9, 7
    A, C, S = rand_problem(rng, m, n, 1)
    ref = np.array(A, dtype=np.float64, order="F")
    for j in range(n - 1):
        x, y = blas.drot(ref[:, j].copy(), ref[:, j + 1].copy(), C[j, 0], S[j, 0])
        ref[:, j], ref[:, j + 1] = x, y
    apply(A, C, S)
    e = relerr(A, ref)
    assert e <= 1e-15, f"drot comparison: rel err {e:.3e}"


def pin_swap_closed_form(apply):
    """P-4: c = 0, s = 1 shifts the columns left cyclically; the wrapped
    column picks up the factor (-1)^(n-1).  Exact in binary64."""
    rng = np.random.Generator(np.random.PCG64(105))
    for (m, n, k) in [(4, 5, 3), (3, 6, 7), (2, 2, 3)]:
        A0 = rng.standard_normal((m, n))
        ref = A0.copy()
        for _ in range(k):
            first = ref[:, 0].copy()
            ref[:, :-1] = ref[:, 1:]
            ref[:, -1] = first * (-1.0) ** (n - 1)
        A = colmajor(A0)
        C = colmajor(np.zeros((n - 1, k)))
        S = colmajor(np.ones((n - 1, k)))
        apply(A, C, S)
        assert np.array_equal(np.asarray(A), ref), f"swap closed form m={m} n={n} k={k}"


def pin_n2_composition(apply):
    """P-5: with n = 2 the k rotations compose into one rotation by sum(theta)."""
    rng = np.random.Generator(np.random.PCG64(106))
    m, k = 6, 9
    th = rng.uniform(0, 2 * math.pi, k)
    A0 = rng.standard_normal((m, 2))
    T = float(np.sum(th))
    c, s = math.cos(T), math.sin(T)
    ref = np.stack([c * A0[:, 0] + s * A0[:, 1], -s * A0[:, 0] + c * A0[:, 1]], axis=1)
    A = colmajor(A0)
    apply(A, colmajor(np.cos(th)[None, :]), colmajor(np.sin(th)[None, :]))
    e = relerr(A, ref)
    assert e <= 20 * k * U, f"n=2 composition: rel err {e:.3e}"


def pin_identity_and_reflection(apply):
    """P-6: (c, s) = (1, 0) leaves A unchanged; (c, s) = (-1, 0) negates both
    columns of every pair, so only columns 0 and n-1 change, by (-1)^k."""
    rng = np.random.Generator(np.random.PCG64(107))
    m, n, k = 5, 7, 3
    A0 = rng.standard_normal((m, n))
    A = colmajor(A0)
    apply(A, colmajor(np.ones((n - 1, k))), colmajor(np.zeros((n - 1, k))))
    assert np.array_equal(np.asarray(A), A0), "identity rotations changed A"
    A = colmajor(A0)
    apply(A, colmajor(-np.ones((n - 1, k))), colmajor(np.zeros((n - 1, k))))
    ref = A0.copy()
    ref[:, 0] *= (-1.0) ** k
    ref[:, n - 1] *= (-1.0) ** k
    assert np.array_equal(np.asarray(A), ref), "reflection closed form"


def pin_norm_invariants(apply):
    """P-7: orthogonal transforms keep every row's 2-norm."""
    rng = np.random.Generator(np.random.PCG64(108))
    m, n, k = 20, 33, 17
    A, C, S = rand_problem(rng, m, n, k)
    before = np.linalg.norm(np.asarray(A), axis=1)
    apply(A, C, S)
    after = np.linalg.norm(np.asarray(A), axis=1)
    dev = np.max(np.abs(after - before) / before)
    assert dev <= 6 * U * (n - 1) * k, f"row norm deviation {dev:.3e}"
    assert relerr(np.asarray(A), np.zeros_like(np.asarray(A))) > 0


def pin_round_trip(apply):
    """P-8: the inverse sequence recovers A."""
    rng = np.random.Generator(np.random.PCG64(109))
    m, n, k = 11, 17, 6
    A, C, S = rand_problem(rng, m, n, k, lda=13)
    A0 = np.array(A)
    apply(A, C, S)
    assert relerr(A, A0) > 1e-3, "forward sequence did nothing"
    apply(A, C, S, inverse=True)
    e = relerr(A, A0)
    assert e <= 12 * U * (n - 1) * k, f"round trip rel err {e:.3e}"


def pin_row_independence(apply):
    """P-9: permuting or subsetting rows permutes/subsets the output bitwise."""
    rng = np.random.Generator(np.random.PCG64(110))
    m, n, k = 12, 10, 5
    A, C, S = rand_problem(rng, m, n, k)
    A0 = np.array(A)
    apply(A, C, S)
    full = np.array(A)
    perm = rng.permutation(m)
    B = colmajor(A0[perm])
    apply(B, C, S)
    assert np.array_equal(np.asarray(B), full[perm]), "row permutation not bitwise"
    sub = np.sort(rng.choice(m, 4, replace=False))
    B = colmajor(A0[sub])
    apply(B, C, S)
    assert np.array_equal(np.asarray(B), full[sub]), "row subset not bitwise"


def load_golden(name):
    """Parse a golden fixture: 'key: v1 v2 ...' lines; '#' starts a comment."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, vals = line.split(":", 1)
            out[key.strip()] = [Fraction(v) for v in vals.split()]
    return out


def pin_hand_worked(apply):
    """A hand-worked example (tests/golden/hand_worked_rotseq.txt)."""
    g = load_golden("hand_worked_rotseq.txt")
    m, n, k = (int(v) for v in g["shape"])
    A0 = np.array([float(v) for v in g["A"]]).reshape(n, m).T
    C = np.array([float(v) for v in g["C"]]).reshape(k, n - 1).T
    S = np.array([float(v) for v in g["S"]]).reshape(k, n - 1).T
    ref = np.array([float(v) for v in g["result"]]).reshape(n, m).T
    A = colmajor(A0)
    apply(A, colmajor(C), colmajor(S))
    e = relerr(A, ref)
    assert e <= 8 * U * (n - 1) * k, f"hand-worked example: rel err {e:.3e}"


ALL_PINS = [
    pin_dense_bruteforce,
    pin_inverse_dense,
    pin_exact_rational,
    pin_drot,
    pin_swap_closed_form,
    pin_n2_composition,
    pin_identity_and_reflection,
    pin_norm_invariants,
    pin_round_trip,
    pin_row_independence,
    pin_hand_worked,
]


# ------------------------------------------------- left application pins
#
# Each takes ``apply_left(A, C, S, inverse=False)``: rotations mixing the
# adjacent rows j, j+1 of A with the per-pair formula of Algorithm 1, in the
# order of Algorithm 2; C and S are (m-1) x k.  In matrix form A <- Q^T A
# (Q the m x m product of the G(j,p) as above), and Q A for the inverse.

def pin_left_dense(apply_left):
    """L-1: Q^T A and Q A computed densely (m != n, padded leading dims)."""
    rng = np.random.Generator(np.random.PCG64(201))
    for idx, (m, n, k) in enumerate([(2, 1, 1), (2, 5, 3), (5, 3, 2), (7, 4, 5), (9, 12, 3)]):
        th = rng.uniform(0, 2 * math.pi, (m - 1, k))
        A = colmajor(rng.standard_normal((m, n)), m + idx % 2)
        C, S = colmajor(np.cos(th), m - 1 + idx % 3), colmajor(np.sin(th))
        Q = dense_q(np.asarray(C), np.asarray(S), m)
        A0 = np.array(A)
        pad = _padding(A)
        apply_left(A, C, S)
        e = relerr(A, Q.T @ A0)
        assert e <= 1e-14, f"left vs dense m={m} n={n} k={k}: rel err {e:.3e}"
        assert np.array_equal(_padding(A), pad), "padding rows of A were modified"
        apply_left(A, C, S, inverse=True)
        e = relerr(A, A0)
        assert e <= 1e-14, f"left round trip m={m} n={n} k={k}: rel err {e:.3e}"
        B = colmajor(A0)
        apply_left(B, C, S, inverse=True)
        e = relerr(B, Q @ A0)
        assert e <= 1e-14, f"left inverse vs dense m={m} n={n} k={k}: rel err {e:.3e}"


def pin_left_is_right_on_transpose(apply_left, apply_right):
    """L-2: rotating rows of A is rotating columns of A^T with the same
    per-pair formula, entry for entry, so the two agree bitwise (ties the
    left application to the pinned right application)."""
    rng = np.random.Generator(np.random.PCG64(202))
    for (m, n, k) in [(6, 4, 3), (13, 9, 7), (2, 3, 4)]:
        th = rng.uniform(0, 2 * math.pi, (m - 1, k))
        A0 = rng.standard_normal((m, n))
        C, S = colmajor(np.cos(th)), colmajor(np.sin(th))
        A = colmajor(A0)
        apply_left(A, C, S)
        T = colmajor(A0.T.copy())
        apply_right(T, C, S)
        assert np.array_equal(np.asarray(A), np.asarray(T).T), f"left != right on A^T m={m} n={n}"


def pin_left_column_norms(apply_left):
    """L-3: rotations from the left keep every column's 2-norm; the rows
    swap closed form c = 0, s = 1 shifts rows up cyclically with the wrapped
    row picking up (-1)^(m-1) per sequence."""
    rng = np.random.Generator(np.random.PCG64(203))
    m, n, k = 21, 8, 11
    th = rng.uniform(0, 2 * math.pi, (m - 1, k))
    A = colmajor(rng.standard_normal((m, n)))
    before = np.linalg.norm(np.asarray(A), axis=0)
    apply_left(A, colmajor(np.cos(th)), colmajor(np.sin(th)))
    dev = np.max(np.abs(np.linalg.norm(np.asarray(A), axis=0) - before) / before)
    assert dev <= 6 * U * (m - 1) * k, f"column norm deviation {dev:.3e}"
    m, n, k = 5, 3, 2
    A0 = rng.standard_normal((m, n))
    ref = A0.copy()
    for _ in range(k):
        first = ref[0].copy()
        ref[:-1] = ref[1:]
        ref[-1] = first * (-1.0) ** (m - 1)
    A = colmajor(A0)
    apply_left(A, colmajor(np.zeros((m - 1, k))), colmajor(np.ones((m - 1, k))))
    assert np.array_equal(np.asarray(A), ref), "left swap closed form"


LEFT_PINS = [pin_left_dense, pin_left_column_norms]


# ------------------------------------------------------- reflector pins
#
# Each takes ``apply_refl(A, TAU, NU, inverse=False, left=False)``.  The
# reflector (j, p) is H = I - tau v v^T with v = e_j + nu e_{j+1}.

def dense_h(TAU, NU, n):
    """prod_p prod_j H(j, p) in Algorithm 2's order, as a dense matrix."""
    Q = np.eye(n)
    nm1, k = TAU.shape
    for p in range(k):
        for j in range(nm1):
            v = np.zeros(n)
            v[j] = 1.0
            v[j + 1] = NU[j, p]
            Q = Q @ (np.eye(n) - TAU[j, p] * np.outer(v, v))
    return Q


def orthogonal_reflectors(rng, r, k):
    """tau = 2 / (1 + nu^2): every H is orthogonal (a true reflection)."""
    nu = rng.standard_normal((r, k)) * rng.choice([0.1, 1.0, 10.0], (r, k))
    return 2.0 / (1.0 + nu * nu), nu


def pin_refl_dense(apply_refl):
    """R-1: A H(0,0)...H(n-2,k-1) densely, for orthogonal and for arbitrary
    (tau, nu) (the formula is applied as written either way); the reverse
    order densely; rows from the left as (prod H)^T A."""
    rng = np.random.Generator(np.random.PCG64(301))
    for idx, (m, n, k) in enumerate([(1, 2, 1), (4, 3, 2), (5, 7, 3), (3, 9, 4)]):
        for ortho in (True, False):
            if ortho:
                tau, nu = orthogonal_reflectors(rng, n - 1, k)
            else:
                tau, nu = rng.uniform(-0.5, 2.5, (n - 1, k)), rng.standard_normal((n - 1, k))
            A0 = rng.standard_normal((m, n))
            H = dense_h(tau, nu, n)
            A = colmajor(A0, m + idx % 2)
            pad = _padding(A)
            apply_refl(A, colmajor(tau, n - 1 + idx % 3), colmajor(nu))
            e = relerr(A, A0 @ H)
            assert e <= 1e-13, f"reflectors vs dense m={m} n={n} k={k} ortho={ortho}: {e:.3e}"
            assert np.array_equal(_padding(A), pad), "padding rows of A were modified"
            Hr = np.eye(n)
            for p in reversed(range(k)):
                for j in reversed(range(n - 1)):
                    v = np.zeros(n)
                    v[j], v[j + 1] = 1.0, nu[j, p]
                    Hr = Hr @ (np.eye(n) - tau[j, p] * np.outer(v, v))
            A = colmajor(A0)
            apply_refl(A, colmajor(tau), colmajor(nu), inverse=True)
            e = relerr(A, A0 @ Hr)
            assert e <= 1e-13, f"reverse reflectors vs dense m={m} n={n} k={k}: {e:.3e}"
            B0 = rng.standard_normal((n, m))
            B = colmajor(B0)
            apply_refl(B, colmajor(tau), colmajor(nu), left=True)
            e = relerr(B, H.T @ B0)
            assert e <= 1e-13, f"left reflectors vs dense n={n} k={k}: {e:.3e}"


def pin_refl_norm_transfer(apply_refl):
    """R-2: reflectors built from the row itself push its whole norm into the
    last column.  For the pair (x, y), nu = (y + sign(y) r) / x with
    r = hypot(x, y) and tau = 2 / (1 + nu^2) solve [x y] H = [0, +-r]
    (a root of x nu^2 - 2 y nu - x = 0); x = 0 needs tau = 0."""
    rng = np.random.Generator(np.random.PCG64(302))
    n = 9
    row = rng.standard_normal(n)
    row[0] = 0.0  # the first pair needs no reflection: tau = 0
    tau, nu = np.zeros((n - 1, 1)), np.zeros((n - 1, 1))
    x = row.copy()
    for j in range(n - 1):
        a, b = x[j], x[j + 1]
        r = math.hypot(a, b)
        if a == 0.0:
            t, v = 0.0, 0.0
        else:
            v = (b + math.copysign(r, b)) / a
            t = 2.0 / (1.0 + v * v)
        tau[j, 0], nu[j, 0] = t, v
        # exact image of the pair under H (the orthogonal reflector maps it to (0, +-r))
        x[j], x[j + 1] = 0.0, (-math.copysign(r, b) if a != 0.0 else b)
    A = colmajor(row[None, :])
    apply_refl(A, colmajor(tau), colmajor(nu))
    out = np.asarray(A)[0]
    nrm = float(np.linalg.norm(row))
    assert np.max(np.abs(out[:-1])) <= 40 * n * U * nrm, f"entries not annihilated: {out[:-1]}"
    assert abs(out[-1] - x[-1]) <= 40 * n * U * nrm, f"last entry {out[-1]} != {x[-1]}"


def pin_refl_closed_forms(apply_refl):
    """R-3: tau = 0 is the identity (bitwise); (tau, nu) = (2, 0) is
    diag(-1, 1) on the pair, so one sequence negates columns 0..n-2 once each
    and k sequences multiply them by (-1)^k (exact); orthogonal reflectors
    keep row norms and the reverse order undoes the forward order."""
    rng = np.random.Generator(np.random.PCG64(303))
    m, n, k = 4, 6, 3
    A0 = rng.standard_normal((m, n))
    A = colmajor(A0)
    apply_refl(A, colmajor(np.zeros((n - 1, k))), colmajor(rng.standard_normal((n - 1, k))))
    assert np.array_equal(np.asarray(A), A0), "tau = 0 changed A"
    A = colmajor(A0)
    apply_refl(A, colmajor(np.full((n - 1, k), 2.0)), colmajor(np.zeros((n - 1, k))))
    ref = A0.copy()
    ref[:, :-1] *= (-1.0) ** k
    assert np.array_equal(np.asarray(A), ref), "(tau, nu) = (2, 0) closed form"
    m, n, k = 9, 23, 8
    tau, nu = orthogonal_reflectors(rng, n - 1, k)
    A0 = rng.standard_normal((m, n))
    A = colmajor(A0)
    apply_refl(A, colmajor(tau), colmajor(nu))
    dev = np.max(np.abs(np.linalg.norm(np.asarray(A), axis=1) / np.linalg.norm(A0, axis=1) - 1))
    assert dev <= 40 * U * (n - 1) * k, f"row norm deviation {dev:.3e}"
    assert relerr(np.asarray(A), A0) > 1e-3
    apply_refl(A, colmajor(tau), colmajor(nu), inverse=True)
    e = relerr(A, A0)
    assert e <= 40 * U * (n - 1) * k, f"reflector round trip {e:.3e}"


REFL_PINS = [pin_refl_dense, pin_refl_norm_transfer, pin_refl_closed_forms]


# ---------------------------------------------------------------------------
# Sequences of 3x3 reflectors (the double-shift QR case named in Section 9).
# Reflector (j, p) is I - tau v v^T with v = e_j + nu1 e_{j+1} + nu2 e_{j+2};
# apply_refl3(A, TAU, NU1, NU2) applies A <- A H(0,0) ... H(n-3,k-1) in place.

def dense_h3(TAU, NU1, NU2, n):
    """Product H(0,0) H(1,0) ... H(n-3,k-1) as a dense n x n matrix."""
    H = np.eye(n)
    for p in range(TAU.shape[1]):
        for j in range(n - 2):
            v = np.zeros(n)
            v[j], v[j + 1], v[j + 2] = 1.0, NU1[j, p], NU2[j, p]
            H = H @ (np.eye(n) - TAU[j, p] * np.outer(v, v))
    return H


def orthogonal_reflectors3(rng, r, k):
    """Orthogonal 3x3 reflectors: tau = 2 / (1 + nu1^2 + nu2^2), 10% tau = 0."""
    nu1, nu2 = rng.standard_normal((r, k)), rng.standard_normal((r, k))
    tau = 2.0 / (1.0 + nu1 * nu1 + nu2 * nu2)
    tau[rng.random((r, k)) < 0.1] = 0.0
    return tau, nu1, nu2


def pin_refl3_dense(apply_refl3):
    """R3-1: A H(0,0)...H(n-3,k-1) against the dense product, for orthogonal
    and for arbitrary (tau, nu1, nu2), with padded leading dimensions."""
    rng = np.random.Generator(np.random.PCG64(311))
    for idx, (m, n, k) in enumerate([(1, 3, 1), (4, 3, 2), (5, 4, 3), (3, 7, 4), (6, 10, 2)]):
        for ortho in (True, False):
            if ortho:
                tau, nu1, nu2 = orthogonal_reflectors3(rng, n - 2, k)
            else:
                tau = rng.uniform(-0.5, 2.5, (n - 2, k))
                nu1, nu2 = rng.standard_normal((n - 2, k)), rng.standard_normal((n - 2, k))
            A0 = rng.standard_normal((m, n))
            A = colmajor(A0, m + idx % 2)
            pad = _padding(A)
            apply_refl3(A, colmajor(tau, n - 2 + idx % 3), colmajor(nu1, n - 1), colmajor(nu2))
            e = relerr(A, A0 @ dense_h3(tau, nu1, nu2, n))
            assert e <= 1e-13, f"3x3 reflectors vs dense m={m} n={n} k={k} ortho={ortho}: {e:.3e}"
            assert np.array_equal(_padding(A), pad), "padding rows of A were modified"


def pin_refl3_norm_transfer(apply_refl3):
    """R3-2: reflectors built from the row push its whole norm into entry
    n-2.  A Householder reflector maps x = (a, b, c) to y = (0, -sign(b) r, 0),
    r = |x|, when v is proportional to x - y: v = (1, (b + sign(b) r)/a, c/a)
    and tau = 2 / v^T v.  The next window starts with the entry just written,
    so a stays nonzero; the final row is zero except entry n-2 = +-|row|."""
    rng = np.random.Generator(np.random.PCG64(312))
    n = 11
    row = rng.standard_normal(n)
    tau, nu1, nu2 = np.zeros((n - 2, 1)), np.zeros((n - 2, 1)), np.zeros((n - 2, 1))
    x = row.copy()
    for j in range(n - 2):
        a, b, c = x[j], x[j + 1], x[j + 2]
        r = math.sqrt(a * a + b * b + c * c)
        v1, v2 = (b + math.copysign(r, b)) / a, c / a
        tau[j, 0], nu1[j, 0], nu2[j, 0] = 2.0 / (1.0 + v1 * v1 + v2 * v2), v1, v2
        x[j], x[j + 1], x[j + 2] = 0.0, -math.copysign(r, b), 0.0
    A = colmajor(row[None, :])
    apply_refl3(A, colmajor(tau), colmajor(nu1), colmajor(nu2))
    out = np.asarray(A)[0]
    nrm = float(np.linalg.norm(row))
    rest = np.delete(out, n - 2)
    assert np.max(np.abs(rest)) <= 40 * n * U * nrm, f"entries not annihilated: {rest}"
    assert abs(out[n - 2] - x[n - 2]) <= 40 * n * U * nrm, f"entry n-2 {out[n - 2]} != {x[n - 2]}"
    assert abs(abs(x[n - 2]) - nrm) <= 40 * n * U * nrm


def pin_refl3_closed_forms(apply_refl3, apply_refl2):
    """R3-3: tau = 0 is the identity (bitwise); (tau, nu1, nu2) = (2, 0, 0) is
    diag(-1, 1, 1) on the window, so k sequences multiply columns 0..n-3 by
    (-1)^k (exact); nu2 = 0 is the 2x2 reflector (tau, nu1) on columns j, j+1
    with the same roundings, so it equals the 2x2 sequence whose last
    reflector is the identity; orthogonal reflectors keep row norms."""
    rng = np.random.Generator(np.random.PCG64(313))
    m, n, k = 4, 7, 3
    A0 = rng.standard_normal((m, n))
    A = colmajor(A0)
    apply_refl3(A, colmajor(np.zeros((n - 2, k))), colmajor(rng.standard_normal((n - 2, k))),
                colmajor(rng.standard_normal((n - 2, k))))
    assert np.array_equal(np.asarray(A), A0), "tau = 0 changed A"
    A = colmajor(A0)
    apply_refl3(A, colmajor(np.full((n - 2, k), 2.0)), colmajor(np.zeros((n - 2, k))),
                colmajor(np.zeros((n - 2, k))))
    ref = A0.copy()
    ref[:, :-2] *= (-1.0) ** k
    assert np.array_equal(np.asarray(A), ref), "(tau, nu1, nu2) = (2, 0, 0) closed form"
    m, n, k = 5, 9, 4
    tau, nu1, _ = orthogonal_reflectors3(rng, n - 2, k)
    A0 = rng.standard_normal((m, n))
    A = colmajor(A0)
    apply_refl3(A, colmajor(tau), colmajor(nu1), colmajor(np.zeros((n - 2, k))))
    B = colmajor(A0)
    apply_refl2(B, colmajor(np.vstack([tau, np.zeros((1, k))])), colmajor(np.vstack([nu1, np.zeros((1, k))])))
    assert np.array_equal(np.asarray(A), np.asarray(B)), "nu2 = 0 differs from the 2x2 reflectors"
    m, n, k = 9, 23, 8
    tau, nu1, nu2 = orthogonal_reflectors3(rng, n - 2, k)
    A0 = rng.standard_normal((m, n))
    A = colmajor(A0)
    apply_refl3(A, colmajor(tau), colmajor(nu1), colmajor(nu2))
    dev = np.max(np.abs(np.linalg.norm(np.asarray(A), axis=1) / np.linalg.norm(A0, axis=1) - 1))
    assert dev <= 40 * U * (n - 2) * k, f"row norm deviation {dev:.3e}"
    assert relerr(np.asarray(A), A0) > 1e-3


REFL3_PINS = [pin_refl3_dense, pin_refl3_norm_transfer]
