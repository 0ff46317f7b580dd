"""GPU parity of the batch path (rotseq_batch_* / rotseq_batched_*) through
the C ABI: every entry against the CPU oracle, bitwise against single calls
of the same kernel, repeated and graph-replayed executions, and the uneven
512-problem batch (n log-uniform in [64, 2048], m = n, k in {8, 16, 32, 64})
on sampled rows.
"""
import numpy as np
import pytest

import oracle
import paper_2412_01852_amd as rs
from paper_2412_01852_amd.inputs import batched_problems, make_problem
from gpu_util import TOL, oracle_rows, relerr, say, to_dev, widened

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.synchronize()


# m, n, k, lda pad: ragged tiles, k not a multiple of the band, n = 2, k > n,
# quick-return entries (m = 0, n = 1, k = 0) mixed in.
MIXED = [(130, 17, 33, 2), (64, 64, 64, 0), (1, 2, 1, 0), (200, 2, 9, 1), (0, 9, 4, 0),
         (70, 300, 8, 0), (9, 1, 5, 0), (65, 40, 0, 0), (3, 129, 128, 1), (257, 100, 16, 3),
         (100, 5, 20, 0), (33, 77, 1, 5)]


def mixed_problems(seed=11):
    return [make_problem(m, n, k, seed=seed + i, lda=max(1, m) + pa)
            for i, (m, n, k, pa) in enumerate(MIXED)]


def upload(pbs, dtype):
    return [(to_dev(p.A, dtype), to_dev(p.C, dtype), to_dev(p.S, dtype)) for p in pbs]


def oracle_full(pb, dtype, times=1):
    ref = oracle.colmajor(widened(pb.A, dtype))
    C, S = oracle.colmajor(widened(pb.C, dtype)), oracle.colmajor(widened(pb.S, dtype))
    for _ in range(times):
        oracle.rotseq(ref, C, S)
    return np.asarray(ref)


def check_status(*batches):
    """No bounded wait gave up: in the device word (plain calls) or in the
    plans' own words (batches)."""
    assert rs.device_status(reset=True) == 0, "a device-side wait timed out"
    for b in batches:
        assert b.status() == (0, [0] * len(b._keep)), "a wait of the batch timed out"


@pytest.mark.parametrize("arith", ["lift", "exact", "fma"])
@pytest.mark.parametrize("waves", [0, 2, 16])
def test_batch_mixed_fp64(arith, waves):
    import torch
    say(f"batch mixed fp64 arith={arith} waves={waves}")
    pbs = mixed_problems()
    dev = upload(pbs, "f64")
    a = {"lift": rs.ARITH_LIFT, "exact": rs.ARITH_EXACT, "fma": rs.ARITH_FMA}[arith]
    with rs.Batch(dev, {"arith": a, "waves": waves}) as b:
        info = b.info()
        assert info["count"] == sum(1 for (m, n, k, _) in MIXED if m > 0 and n > 1 and k > 0)
        b.execute()
        torch.cuda.synchronize()
        check_status(b)
    for pb, (A, _, _) in zip(pbs, dev):
        got = rs.host_colmajor(A)
        ref = oracle_full(pb, "f64")
        if arith == "exact":
            assert np.array_equal(got, ref), f"exact batch entry {pb.m}x{pb.n} k={pb.k}"
        else:
            assert relerr(got, ref, pb.A) <= TOL["f64"]


@pytest.mark.parametrize("band", [4, 6, 8])
def test_batch_bitwise_equals_single_calls(band):
    """Same kernel code per band-wave, so a batch equals single calls bitwise."""
    import torch
    say(f"batch vs single calls band={band}")
    pbs = mixed_problems(seed=40)
    dev_b = upload(pbs, "f64")
    dev_s = upload(pbs, "f64")
    plans = []
    if band == 8:
        rs.batched(dev_b)  # raises on a time-out
    else:
        plans.append(rs.Batch(dev_b, {"band": band}))
        plans[0].execute()
    for A, C, S in dev_s:
        rs.rotseq(A, C, S, opts={"kernel": rs.KERNEL_CHAIN, "band": band})
    torch.cuda.synchronize()
    check_status(*plans)
    for (Ab, _, _), (As, _, _) in zip(dev_b, dev_s):
        assert torch.equal(Ab, As)


def test_batch_fp32():
    import torch
    say("batch mixed fp32")
    pbs = mixed_problems(seed=70)
    dev = upload(pbs, "f32")
    rs.batched(dev)
    torch.cuda.synchronize()
    check_status()
    for pb, (A, _, _) in zip(pbs, dev):
        assert relerr(rs.host_colmajor(A), oracle_full(pb, "f32"), widened(pb.A, "f32")) <= TOL["f32"]


def test_batch_execute_twice_and_tune():
    """Executions compose (A <- A Q twice); tuning keeps results correct."""
    import torch
    say("batch execute twice, then tune")
    pbs = mixed_problems(seed=90)
    dev = upload(pbs, "f64")
    with rs.Batch(dev) as b:
        b.execute()
        b.execute()
        torch.cuda.synchronize()
        check_status(b)
        for pb, (A, _, _) in zip(pbs, dev):
            assert relerr(rs.host_colmajor(A), oracle_full(pb, "f64", times=2), pb.A) <= 2 * TOL["f64"]
        b.tune(reps=1)
        assert b.info()["waves"] in (2, 4, 8, 16)
        before = [rs.host_colmajor(A) for A, _, _ in dev]
        b.execute()
        torch.cuda.synchronize()
        check_status(b)
        for before_i, pb, (A, _, _) in zip(before, pbs, dev):
            ref = oracle.colmajor(before_i)
            oracle.rotseq(ref, oracle.colmajor(pb.C), oracle.colmajor(pb.S))
            assert relerr(rs.host_colmajor(A), np.asarray(ref), pb.A) <= TOL["f64"]


def test_batch_graph_replays_match_eager():
    """Capture one execution into a graph; every replay (with eager work in
    between) must equal an eager execution on a twin copy, bitwise."""
    import torch
    say("batch graph capture and replays")
    pbs = mixed_problems(seed=120)
    dev_g = upload(pbs, "f64")
    dev_e = upload(pbs, "f64")
    bg = rs.Batch(dev_g)
    be = rs.Batch(dev_e)
    bg.execute()  # warm-up outside capture (first launches load code objects)
    be.execute()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bg.execute(stream=s)
    torch.cuda.synchronize()
    for r in range(3):
        g.replay()
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        be.execute()
        torch.cuda.synchronize()
        check_status(bg, be)
        float(junk)
        for (Ag, _, _), (Ae, _, _) in zip(dev_g, dev_e):
            assert torch.equal(Ag, Ae), f"replay {r} differs from eager execution"
    bg.close()
    be.close()


def test_uneven_512_batch_sampled():
    """The 512-problem batch at full size: 24 entries checked on sampled rows
    (oracle per row), the rest for finiteness and norm preservation."""
    import torch
    say("uneven 512-problem batch (seed 4)")
    pbs = batched_problems(512, seed=4)
    dev = upload(pbs, "f64")
    norms0 = [np.linalg.norm(np.asarray(p.A), axis=1) for p in pbs]
    with rs.Batch(dev) as b:
        info = b.info()
        assert info["count"] == 512
        b.execute()
        torch.cuda.synchronize()
        check_status(b)
    rng = np.random.default_rng(0)
    pick = set(rng.choice(512, 24, replace=False).tolist())
    for i, (pb, (A, _, _)) in enumerate(zip(pbs, dev)):
        got = rs.host_colmajor(A)
        assert np.all(np.isfinite(got))
        # rotations preserve every row's 2-norm
        assert np.allclose(np.linalg.norm(got, axis=1), norms0[i], rtol=1e-12, atol=1e-12)
        if i in pick:
            rows = np.sort(rng.choice(pb.m, min(pb.m, 8), replace=False))
            ref = oracle_rows(pb.A, pb.C, pb.S, rows, "f64")
            assert relerr(got[rows], ref, np.asarray(pb.A)[rows]) <= TOL["f64"]


def test_batch_update_pointers():
    """rotseq_batch_update_*: the plan runs on other buffers of the same
    shapes (other leading dimensions too), eagerly and from a captured graph;
    a shape change is refused and leaves the plan as it was."""
    import torch
    say("batch pointer update")
    pbs1 = mixed_problems(seed=150)
    pbs2 = [make_problem(p.m, p.n, p.k, seed=300 + i, lda=max(1, p.m) + (i % 3))
            for i, p in enumerate(pbs1)]
    dev1, dev2 = upload(pbs1, "f64"), upload(pbs2, "f64")
    b = rs.Batch(dev1)
    b.execute()
    b.update(dev2)
    b.execute()
    torch.cuda.synchronize()
    check_status(b)
    for pb, (A, _, _) in zip(pbs1, dev1):
        assert relerr(rs.host_colmajor(A), oracle_full(pb, "f64"), pb.A) <= TOL["f64"]
    for pb, (A, _, _) in zip(pbs2, dev2):
        assert relerr(rs.host_colmajor(A), oracle_full(pb, "f64"), pb.A) <= TOL["f64"]
    # a different k for entry 3 is refused with its index and argument
    bad = list(dev2)
    A3, C3, S3 = bad[3]
    bad[3] = (A3, C3[:, :max(1, C3.shape[1] - 1)].contiguous(), S3[:, :max(1, S3.shape[1] - 1)].contiguous())
    with pytest.raises(rs.RotseqError) as e:
        b.update(bad)
    assert e.value.code == -(1000 * 4 + 3)
    # graph captured on dev2's pointers, then updated back to dev1: replays use dev1
    dev3 = upload(pbs1, "f64")
    b.update(dev3)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            b.execute(stream=s)
    torch.cuda.synchronize()
    dev4 = upload(pbs2, "f64")
    b.update(dev4)
    g.replay()
    torch.cuda.synchronize()
    check_status(b)
    for pb, (A, _, _) in zip(pbs2, dev4):
        assert relerr(rs.host_colmajor(A), oracle_full(pb, "f64"), pb.A) <= TOL["f64"]
    for pb, (A, _, _) in zip(pbs1, dev3):  # untouched by the replay after the update
        assert np.array_equal(rs.host_colmajor(A), np.asarray(pb.A))
    b.close()
