"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar: relative Frobenius error ||A_gpu - A_ref|| / ||A_in|| <= 1e-13 (FP64)
and <= 5e-6 (FP32, oracle in FP64 on the widened FP32 inputs); the exact
arithmetic mode (Algorithm 1 without fused multiply-adds) must be bitwise.
Large shapes are checked on sampled rows, which the oracle computes alone
because rows of A never interact.
"""
import os

import numpy as np
import pytest

import oracle
import paper_2412_01852_amd as rs
from paper_2412_01852_amd.inputs import make_problem
from gpu_util import TOL, oracle_rows, padding_bits, relerr, say, to_dev, widened

pytestmark = pytest.mark.gpu

ARITHS = {"exact": rs.ARITH_EXACT, "fma": rs.ARITH_FMA, "lift": rs.ARITH_LIFT}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.synchronize()


def run_full(pb, dtype, opts=None):
    """Whole-matrix run; returns (gpu result, oracle result, padding ok)."""
    import torch
    A = to_dev(pb.A, dtype)
    C = to_dev(pb.C, dtype)
    S = to_dev(pb.S, dtype)
    pad_before = padding_bits(A)
    rs.rotseq(A, C, S, opts=opts)
    torch.cuda.synchronize()
    assert rs.device_status(reset=True) == 0, "a device-side wait timed out"
    got = rs.host_colmajor(A)
    ref = oracle.colmajor(widened(pb.A, dtype))
    oracle.rotseq(ref, oracle.colmajor(widened(pb.C, dtype)), oracle.colmajor(widened(pb.S, dtype)))
    return got, np.asarray(ref), np.array_equal(pad_before, padding_bits(A))


@pytest.mark.parametrize("arith", sorted(ARITHS))
def test_plain_512_fp64(arith):
    """m = n = 512, k = 32 (the small plain configuration)."""
    say(f"plain 512x512 k=32 fp64 arith={arith}")
    pb = make_problem(512, 512, 32, seed=1)
    got, ref, pad_ok = run_full(pb, "f64", {"arith": ARITHS[arith]})
    assert pad_ok
    if arith == "exact":
        assert np.array_equal(got, ref), "exact mode must be bitwise equal to the oracle"
    else:
        assert relerr(got, ref, pb.A) <= TOL["f64"]


EDGE = [
    # m, n, k, lda pad, ldc pad, lds pad
    (1, 2, 1, 0, 0, 0), (63, 3, 2, 1, 0, 2), (65, 2, 5, 3, 1, 0), (64, 64, 64, 0, 0, 0),
    (130, 17, 33, 2, 3, 1), (100, 5, 20, 0, 0, 0), (70, 40, 17, 6, 0, 0), (1, 300, 3, 0, 0, 0),
    (129, 1, 5, 0, 0, 0), (0, 7, 3, 0, 0, 0), (7, 7, 0, 0, 0, 0), (7, 0, 3, 0, 0, 0),
    (200, 2, 1, 0, 0, 0), (3, 129, 128, 1, 1, 1),
]


@pytest.mark.parametrize("m,n,k,pa,pc,ps", EDGE)
@pytest.mark.parametrize("arith", ["exact", "lift"])
@pytest.mark.parametrize("kernel", ["chain", "multipass"])
def test_edges_fp64(m, n, k, pa, pc, ps, arith, kernel):
    say(f"edge fp64 m={m} n={n} k={k} pads={pa},{pc},{ps} arith={arith} kernel={kernel}")
    pb = make_problem(m, n, k, seed=m + 7 * n + 13 * k,
                      lda=max(1, m) + pa, ldc=max(1, n - 1) + pc, lds=max(1, n - 1) + ps)
    kern = rs.KERNEL_CHAIN if kernel == "chain" else rs.KERNEL_MULTIPASS
    got, ref, pad_ok = run_full(pb, "f64", {"arith": ARITHS[arith], "kernel": kern})
    assert pad_ok, "padding rows of A were modified"
    if arith == "exact":
        assert np.array_equal(got, ref)
    else:
        assert relerr(got, ref, pb.A) <= TOL["f64"]


@pytest.mark.parametrize("band", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("arith", sorted(ARITHS))
def test_multipass_bands_fp64(band, arith):
    say(f"multipass fp64 band={band} arith={arith}")
    pb = make_problem(200, 300, 37, seed=band)
    got, ref, pad_ok = run_full(pb, "f64", {"arith": ARITHS[arith], "band": band,
                                            "kernel": rs.KERNEL_MULTIPASS})
    assert pad_ok
    if arith == "exact":
        assert np.array_equal(got, ref)
    else:
        assert relerr(got, ref, pb.A) <= TOL["f64"]


CHAIN = [
    # band, waves, publish: waves=1 puts every hand-off through A and the
    # device-scope counters; publish=1 publishes after every column.
    (4, 0, 0), (6, 0, 0), (8, 0, 0), (8, 1, 1), (4, 1, 32), (6, 2, 4), (8, 3, 2),
    (4, 5, 8), (6, 16, 0), (8, 16, 1), (4, 7, 64), (2, 0, 0), (2, 3, 4), (2, 16, 1),
]


@pytest.mark.parametrize("band,k,waves", [(2, 8, 8), (4, 8, 8), (4, 16, 4), (8, 32, 8), (2, 3, 2)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_chain_streaming(band, k, waves, dtype):
    """The streaming form (whole chains per workgroup: waves a multiple of
    the band count, at most 8) over ragged tiles and several tiles per
    workgroup, against the oracle."""
    say(f"chain streaming {dtype} band={band} k={k} waves={waves}")
    pb = make_problem(333, 211, k, seed=band * 10 + k, lda=340)
    got, ref, pad_ok = run_full(pb, dtype, {"kernel": rs.KERNEL_CHAIN, "band": band, "waves": waves})
    assert pad_ok
    assert relerr(got, ref, widened(pb.A, dtype)) <= TOL[dtype]


@pytest.mark.parametrize("band,waves,publish", CHAIN)
@pytest.mark.parametrize("arith", ["exact", "lift"])
def test_chain_fp64(band, waves, publish, arith):
    """Chains of band-waves: LDS hand-off inside a workgroup, A plus
    device-scope progress counters across workgroups."""
    say(f"chain fp64 band={band} waves={waves} publish={publish} arith={arith}")
    pb = make_problem(333, 211, 59, seed=band * 100 + waves, lda=340)
    got, ref, pad_ok = run_full(pb, "f64", {"arith": ARITHS[arith], "band": band,
                                            "kernel": rs.KERNEL_CHAIN, "waves": waves,
                                            "publish": publish})
    assert pad_ok
    if arith == "exact":
        assert np.array_equal(got, ref)
    else:
        assert relerr(got, ref, pb.A) <= TOL["f64"]


@pytest.mark.parametrize("m,n,k", [(512, 512, 32), (65, 40, 17), (1, 2, 1), (130, 17, 33)])
@pytest.mark.parametrize("arith", sorted(ARITHS))
def test_fp32(m, n, k, arith):
    say(f"fp32 m={m} n={n} k={k} arith={arith}")
    pb = make_problem(m, n, k, seed=3 + m)
    got, ref, pad_ok = run_full(pb, "f32", {"arith": ARITHS[arith]})
    assert pad_ok
    assert relerr(got, ref, widened(pb.A, "f32")) <= TOL["f32"]


def sample_rows(m, rng, extra=24):
    fixed = {0, 1, 62, 63, 64, 65, m // 2, m - 65, m - 64, m - 1}
    rows = sorted({r for r in fixed if 0 <= r < m} | set(rng.choice(m, extra, replace=False).tolist()))
    return np.asarray(rows)


def run_sampled(m, n, k, seed, dtype, opts=None):
    import torch
    pb = make_problem(m, n, k, seed=seed)
    A = to_dev(pb.A, dtype)
    C = to_dev(pb.C, dtype)
    S = to_dev(pb.S, dtype)
    norms0 = torch.linalg.vector_norm(A.double(), dim=1)
    rs.rotseq(A, C, S, opts=opts)
    torch.cuda.synchronize()
    assert rs.device_status(reset=True) == 0, "a device-side wait timed out"
    norms1 = torch.linalg.vector_norm(A.double(), dim=1)
    rows = sample_rows(m, np.random.Generator(np.random.PCG64(seed)))
    got = A[torch.as_tensor(rows, device=A.device)].double().cpu().numpy()
    ref = oracle_rows(pb.A, pb.C, pb.S, rows, dtype)
    a0 = widened(pb.A, dtype)[rows]
    drift = float(torch.max(torch.abs(norms1 - norms0) / norms0))
    return relerr(got, ref, a0), drift


def oracle_threads():
    """Host threads for the full-size oracle: the CPU share of one GPU."""
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


def run_full_large(m, n, k, seed, dtype):
    """The default call (the bench's launch configuration) on a full-size
    problem, compared element by element with the threaded oracle (bitwise
    equal to the serial one: rows never interact).  Returns the relative
    error and the largest relative change of a row norm."""
    import torch
    pb = make_problem(m, n, k, seed=seed)
    A = to_dev(pb.A, dtype)
    C = to_dev(pb.C, dtype)
    S = to_dev(pb.S, dtype)
    norms0 = torch.linalg.vector_norm(A.double(), dim=1)
    rs.rotseq(A, C, S)
    torch.cuda.synchronize()
    assert rs.device_status(reset=True) == 0, "a device-side wait timed out"
    norms1 = torch.linalg.vector_norm(A.double(), dim=1)
    drift = float(torch.max(torch.abs(norms1 - norms0) / norms0))
    got = rs.host_colmajor(A)
    del A
    a0 = widened(pb.A, dtype)
    ref = oracle.colmajor(a0)
    oracle.rotseq(ref, oracle.colmajor(widened(pb.C, dtype)), oracle.colmajor(widened(pb.S, dtype)),
                  threads=oracle_threads())
    return relerr(got, np.asarray(ref), a0), drift


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_target_10240_k192_full(dtype):
    """m = n = 10240, k = 192 in the default launch: every element against
    the oracle; every row's norm is preserved (an orthogonal transform)."""
    say(f"target 10240x10240 k=192 {dtype} (all elements)")
    err, drift = run_full_large(10240, 10240, 192, 2, dtype)
    say(f"  rel err {err:.3e}  max row-norm drift {drift:.3e}")
    assert err <= TOL[dtype]
    assert drift <= (1e-12 if dtype == "f64" else 1e-4)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_target_10240_k192_multipass_sampled(dtype):
    """The multipass kernel at the target size on sampled rows."""
    say(f"target 10240x10240 k=192 {dtype} kernel=multipass (sampled rows)")
    err, drift = run_sampled(10240, 10240, 192, 2, dtype, {"kernel": rs.KERNEL_MULTIPASS})
    say(f"  rel err {err:.3e}  max row-norm drift {drift:.3e}")
    assert err <= TOL[dtype]
    assert drift <= (1e-12 if dtype == "f64" else 1e-4)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("k", [1, 8, 32, 128])
def test_tall_32768x4096_full(k, dtype):
    """The tall configuration (memory-bound to compute-bound as k grows) in
    the default launch, every element against the oracle."""
    say(f"tall 32768x4096 k={k} {dtype} (all elements)")
    err, drift = run_full_large(32768, 4096, k, 3 + k, dtype)
    say(f"  rel err {err:.3e}  max row-norm drift {drift:.3e}")
    assert err <= TOL[dtype]
    assert drift <= (1e-12 if dtype == "f64" else 1e-4)


def test_caller_workspace_and_stream():
    """rotseq_ex_d with a caller workspace on a side stream equals the pooled call."""
    import torch
    say("caller workspace + side stream")
    pb = make_problem(300, 257, 40, seed=9)
    A1, C, S = to_dev(pb.A, "f64"), to_dev(pb.C, "f64"), to_dev(pb.S, "f64")
    A2 = to_dev(pb.A, "f64")
    rs.rotseq(A1, C, S)
    nbytes = rs.workspace_bytes("float64", 300, 257, 40)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        rs.rotseq(A2, C, S, opts={"arith": 0}, workspace=ws, stream=side)
    side.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(A1, A2)
    with pytest.raises(rs.RotseqError):
        rs.rotseq(A2, C, S, opts={}, workspace=ws[: nbytes // 2])


def test_repeated_calls_reuse_pool():
    """Back-to-back calls of growing and shrinking size through the pool."""
    import torch
    say("repeated calls")
    for (m, n, k) in [(64, 50, 3), (256, 700, 70), (64, 50, 3), (1000, 33, 5)]:
        pb = make_problem(m, n, k, seed=m + n + k)
        got, ref, _ = run_full(pb, "f64")
        assert relerr(got, ref, pb.A) <= TOL["f64"]
    torch.cuda.synchronize()


@pytest.mark.parametrize("band", [4, 8])
@pytest.mark.parametrize("arith", ["lift", "fma"])
def test_chain_bitwise_equals_multipass(band, arith):
    """Both kernels apply, per element, the same FMAs in the same order (the
    chain kernel's two-step interleave included), so they agree bitwise."""
    import torch
    say(f"chain vs multipass bitwise band={band} arith={arith}")
    pb = make_problem(300, 700, 37, seed=5 + band)
    outs = []
    for kern in (rs.KERNEL_CHAIN, rs.KERNEL_MULTIPASS):
        A = to_dev(pb.A, "f64")
        rs.rotseq(A, to_dev(pb.C, "f64"), to_dev(pb.S, "f64"),
                  opts={"kernel": kern, "band": band, "arith": ARITHS[arith]})
        torch.cuda.synchronize()
        outs.append(A)
    assert rs.device_status(reset=True) == 0
    assert torch.equal(outs[0], outs[1])


INVERSE = [(130, 17, 33, 2, 3, 1), (64, 64, 64, 0, 0, 0), (1, 2, 1, 0, 0, 0), (200, 2, 9, 1, 0, 0),
           (3, 129, 128, 1, 1, 1), (257, 300, 20, 3, 0, 0)]


@pytest.mark.parametrize("m,n,k,pa,pc,ps", INVERSE)
@pytest.mark.parametrize("arith", ["exact", "lift"])
@pytest.mark.parametrize("kernel", ["chain", "multipass"])
def test_inverse_fp64(m, n, k, pa, pc, ps, arith, kernel):
    """opts.inverse applies A <- A Q^T: against the oracle's inverse (bitwise
    in exact mode) and as the undo of a forward call."""
    import torch
    say(f"inverse fp64 m={m} n={n} k={k} arith={arith} kernel={kernel}")
    pb = make_problem(m, n, k, seed=3 * m + n + k,
                      lda=max(1, m) + pa, ldc=max(1, n - 1) + pc, lds=max(1, n - 1) + ps)
    kern = rs.KERNEL_CHAIN if kernel == "chain" else rs.KERNEL_MULTIPASS
    A = to_dev(pb.A, "f64")
    C, S = to_dev(pb.C, "f64"), to_dev(pb.S, "f64")
    pad_before = padding_bits(A)
    rs.rotseq(A, C, S, opts={"arith": ARITHS[arith], "kernel": kern, "inverse": 1})
    torch.cuda.synchronize()
    assert rs.device_status(reset=True) == 0
    assert np.array_equal(pad_before, padding_bits(A))
    got = rs.host_colmajor(A)
    ref = oracle.colmajor(np.asarray(pb.A))
    oracle.rotseq(ref, oracle.colmajor(pb.C), oracle.colmajor(pb.S), inverse=True)
    ref = np.asarray(ref)
    if arith == "exact":
        assert np.array_equal(got, ref), "exact inverse must equal the oracle's inverse loop bitwise"
    else:
        assert relerr(got, ref, pb.A) <= TOL["f64"]
    # forward then inverse recovers A
    rs.rotseq(A, C, S, opts={"arith": ARITHS[arith], "kernel": kern})
    torch.cuda.synchronize()
    assert relerr(rs.host_colmajor(A), np.asarray(pb.A), pb.A) <= 2 * TOL["f64"]


def test_inverse_target_sampled():
    """Inverse at 10240^2, k = 192 in the bench's launch shape, sampled rows."""
    import torch
    say("inverse 10240^2 k=192 sampled rows")
    pb = make_problem(10240, 10240, 192, seed=2)
    A = to_dev(pb.A, "f64")
    rs.rotseq(A, to_dev(pb.C, "f64"), to_dev(pb.S, "f64"), opts={"inverse": 1})
    torch.cuda.synchronize()
    assert rs.device_status(reset=True) == 0
    rows = np.array([0, 1, 63, 64, 5000, 10238, 10239])
    sub = oracle.colmajor(np.asarray(pb.A)[rows])
    oracle.rotseq(sub, oracle.colmajor(pb.C), oracle.colmajor(pb.S), inverse=True)
    got = rs.host_colmajor(A)[rows]
    assert relerr(got, np.asarray(sub), np.asarray(pb.A)[rows]) <= TOL["f64"]
