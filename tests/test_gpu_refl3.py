"""GPU parity of sequences of 3x3 reflectors (rotseq_refl3_*) through the C
ABI against the CPU oracle's loop: ragged row tiles, padded leading
dimensions, k not a multiple of the band, several launches of waves,
arbitrary (non-orthogonal) parameters, FP32, quick returns, a caller
workspace, and the 10240^2, k = 192 size on sampled rows.
"""
import numpy as np
import pytest

import oracle
import paper_2412_01852_amd as rs
from paper_2412_01852_amd.inputs import make_refl3_problem
from gpu_util import TOL, padding_bits, relerr, say, to_dev, widened

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.synchronize()


def _oracle(pb, dtype, rows=None):
    A = widened(pb.A, dtype)
    ref = oracle.colmajor(A if rows is None else A[rows])
    oracle.refl3seq(ref, *(oracle.colmajor(widened(X, dtype)) for X in (pb.TAU, pb.NU1, pb.NU2)))
    return np.asarray(ref)


def _run(pb, dtype, workspace=None):
    import torch
    A = to_dev(pb.A, dtype)
    coef = [to_dev(X, dtype) for X in (pb.TAU, pb.NU1, pb.NU2)]
    pad = padding_bits(A)
    rs.refl3seq(A, *coef, workspace=workspace)
    torch.cuda.synchronize()
    assert np.array_equal(pad, padding_bits(A)), "padding rows of A were modified"
    return A


# m x n, k, padding of lda and of the three coefficient arrays: one tile,
# ragged tiles, n = 3 (one reflector per sequence), n below the prefetch
# depth, k below / at / above one band, 17 bands (two launches), 40 bands
# (three launches), a thin and a wide matrix.
SHAPES = [(64, 64, 8, 0, 0), (130, 37, 13, 3, 1), (1, 3, 1, 0, 0), (70, 3, 20, 0, 2),
          (65, 9, 16, 1, 0), (200, 50, 136, 0, 0), (129, 45, 320, 2, 3), (3000, 20, 24, 0, 0),
          (8, 700, 40, 0, 0), (257, 260, 96, 5, 0)]


@pytest.mark.parametrize("m,n,k,pa,pc", SHAPES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_refl3_parity(m, n, k, pa, pc, dtype):
    say(f"refl3 {dtype} m={m} n={n} k={k} pa={pa} pc={pc}")
    r = max(n - 2, 1)
    pb = make_refl3_problem(m, n, k, seed=11 * m + n + k, lda=m + pa,
                            lds=(r + pc, r, r + 2 * pc))
    A = _run(pb, dtype)
    assert relerr(rs.host_colmajor(A), _oracle(pb, dtype), pb.A) <= TOL[dtype]


def test_refl3_arbitrary_parameters():
    """The formula is applied as written: non-orthogonal (tau, nu1, nu2)."""
    say("refl3 arbitrary parameters")
    m, n, k = 100, 41, 11
    pb = make_refl3_problem(m, n, k, seed=5)
    rng = np.random.Generator(np.random.PCG64(6))
    pb.TAU[...] = rng.uniform(-0.2, 0.2, pb.TAU.shape)
    pb.NU1[...] = rng.standard_normal(pb.NU1.shape)
    pb.NU2[...] = rng.standard_normal(pb.NU2.shape)
    A = _run(pb, "f64")
    ref = _oracle(pb, "f64")
    assert np.linalg.norm(rs.host_colmajor(A) - ref) <= TOL["f64"] * np.linalg.norm(ref)


def test_refl3_identity_and_quick_returns():
    """tau = 0 everywhere leaves A bitwise; n <= 2, m = 0, k = 0 launch nothing."""
    import torch
    say("refl3 identity / quick returns")
    pb = make_refl3_problem(77, 30, 20, seed=9)
    pb.TAU[...] = 0.0
    A = _run(pb, "f64")
    assert np.array_equal(rs.host_colmajor(A), np.asarray(pb.A))
    for m, n, k in [(5, 2, 3), (0, 9, 3), (5, 9, 0), (4, 1, 2)]:
        A = torch.ones((m, n), dtype=torch.float64, device="cuda").t().contiguous().t() if m and n else \
            torch.empty((m, n), dtype=torch.float64, device="cuda")
        r = max(n - 2, 0)
        z = torch.zeros((k, r), dtype=torch.float64, device="cuda").t()  # column-major (r, k)
        rs.refl3seq(A, z, z, z)
        torch.cuda.synchronize()
        if A.numel():
            assert bool((A == 1).all())


def test_refl3_caller_workspace():
    """A caller workspace of the reported size gives the pooled result bitwise;
    one byte less is refused."""
    import torch
    say("refl3 caller workspace")
    pb = make_refl3_problem(150, 90, 30, seed=12)
    ref = rs.host_colmajor(_run(pb, "f64"))
    need = rs.refl3_workspace_bytes("float64", 150, 90, 30)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    assert np.array_equal(rs.host_colmajor(_run(pb, "f64", workspace=ws)), ref)
    small = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    A = to_dev(pb.A, "f64")
    with pytest.raises(rs.RotseqError):
        rs.refl3seq(A, *(to_dev(X, "f64") for X in (pb.TAU, pb.NU1, pb.NU2)), workspace=small)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_refl3_full_size_sampled_rows(dtype):
    """10240 x 10240, k = 192 in the bench's launch configuration: rows are
    independent, so the oracle computes a sample of rows (first, last, and
    across tiles) exactly."""
    say(f"refl3 full size 10240x10240 k=192 {dtype}")
    m = n = 10240
    k = 192
    pb = make_refl3_problem(m, n, k, seed=3)
    A = _run(pb, dtype)
    rows = np.array([0, 1, 63, 64, 4097, 7777, m - 65, m - 1])
    got = A[torch_index(rows)].detach().cpu().to(dtype=__import__("torch").float64).numpy()
    ref = _oracle(pb, dtype, rows)
    assert relerr(got, ref, widened(pb.A, dtype)[rows]) <= TOL[dtype]


def torch_index(rows):
    import torch
    return torch.as_tensor(rows, device="cuda")


# Inverse order and application from the left (rotseq_refl3_ex_*): m x n, k,
# lda padding; ragged tiles, one tile, three rows, several launches.
SIDE_SHAPES = [(130, 37, 13, 3), (64, 64, 8, 0), (3, 70, 5, 1), (257, 260, 96, 5), (65, 9, 16, 1),
               (40, 3, 20, 0)]


def _side_problem(m, n, k, pa, left, seed):
    """A (m x n, lda = m + pa) and reflectors over the mixed dimension."""
    r = m if left else n
    A = make_refl3_problem(m, n, 1, seed=seed, lda=m + pa).A
    R = make_refl3_problem(1, r, k, seed=seed + 1)
    return A, (R.TAU, R.NU1, R.NU2)


@pytest.mark.parametrize("m,n,k,pa", SIDE_SHAPES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("inverse,left", [(True, False), (False, True), (True, True)])
def test_refl3_inverse_and_left(m, n, k, pa, dtype, inverse, left):
    import torch
    say(f"refl3 {dtype} m={m} n={n} k={k} inverse={inverse} left={left}")
    r = m if left else n
    A0, coef = _side_problem(m, n, k, pa, left, seed=7 * m + n + k)
    A = to_dev(A0, dtype)
    dcoef = [to_dev(X, dtype) for X in coef]
    pad = padding_bits(A)
    rs.refl3seq(A, *dcoef, opts={"inverse": int(inverse), "left": int(left)})
    torch.cuda.synchronize()
    assert np.array_equal(pad, padding_bits(A)), "padding rows of A were modified"
    ref = oracle.colmajor(widened(A0, dtype))
    if r > 2:
        oracle.refl3seq(ref, *(oracle.colmajor(widened(X, dtype)) for X in coef),
                        inverse=inverse, left=left)
    err = relerr(rs.host_colmajor(A), np.asarray(ref), A0)
    say(f"  rel err {err:.3e}")
    assert err <= TOL[dtype] * (10 if dtype == "f32" else 1)


@pytest.mark.parametrize("left", [False, True])
def test_refl3_inverse_undoes_forward(left):
    """Orthogonal reflectors: the inverse call undoes a forward call."""
    import torch
    m, n, k = 150, 90, 21
    r = m if left else n
    rng = np.random.default_rng(3)
    NU1, NU2 = rng.standard_normal((r - 2, k)), rng.standard_normal((r - 2, k))
    TAU = 2.0 / (1.0 + NU1 ** 2 + NU2 ** 2)
    A0 = make_refl3_problem(m, n, 1, seed=4).A
    A = to_dev(A0, "f64")
    dcoef = [to_dev(np.asfortranarray(X), "f64") for X in (TAU, NU1, NU2)]
    rs.refl3seq(A, *dcoef, opts={"left": int(left)})
    rs.refl3seq(A, *dcoef, opts={"left": int(left), "inverse": 1})
    torch.cuda.synchronize()
    assert relerr(rs.host_colmajor(A), np.asarray(A0), A0) <= 1e-13


def test_refl3_ex_refuses_other_options():
    A0, coef = _side_problem(70, 40, 8, 0, False, seed=9)
    A = to_dev(A0, "f64")
    dcoef = [to_dev(X, "f64") for X in coef]
    with pytest.raises(rs.RotseqError):
        rs.refl3seq(A, *dcoef, opts={"band": 4})
