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
