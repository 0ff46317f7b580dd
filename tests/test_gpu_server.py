"""GPU parity of the serving path (rotseq_server_*) through the C ABI:
resident matrices swept repeatedly, against the CPU oracle applied sweep by
sweep; admission under a small device budget; a matrix served alone and
amid other traffic gives bitwise the same result; error codes."""
import numpy as np
import pytest

import oracle
import paper_2412_01852_amd as rs
from paper_2412_01852_amd.inputs import make_cs, make_problem
from gpu_util import TOL, relerr, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.synchronize()


SHAPES = [(130, 17), (64, 64), (1, 2), (200, 2), (70, 300), (257, 100), (3, 129)]
KS = [8, 33, 1, 0, 16]


def sweeps_for(i, n, count, seed=0):
    rng = np.random.default_rng(1000 * seed + i)
    return [make_cs(n, KS[(i + s) % len(KS)], rng) for s in range(count)]


def oracle_sweeps(A, sweeps):
    ref = oracle.colmajor(np.asarray(A))
    for C, S in sweeps:
        if C.shape[1] and ref.shape[0] and ref.shape[1] > 1:
            oracle.rotseq(ref, oracle.colmajor(C), oracle.colmajor(S))
    return np.asarray(ref)


def test_server_sweeps_match_oracle():
    say("server: 7 matrices x 4 sweeps")
    pbs = [make_problem(m, n, 1, seed=50 + i) for i, (m, n) in enumerate(SHAPES)]
    plans = [sweeps_for(i, pb.n, 4) for i, pb in enumerate(pbs)]
    with rs.Server() as srv:
        ids = [srv.open(pb.A) for pb in pbs]
        tickets = []
        for s in range(4):  # interleave matrices, keep per-matrix order
            for i, mid in enumerate(ids):
                C, S = plans[i][s]
                tickets.append(srv.submit(mid, C, S))
        for t in tickets:
            rc, info = srv.wait(t)
            assert rc == 0
            assert info["submit_us"] <= info["start_us"] <= info["end_us"]
        for i, (pb, mid) in enumerate(zip(pbs, ids)):
            got = srv.read(mid, pb.m, pb.n)
            ref = oracle_sweeps(pb.A, plans[i])
            assert relerr(got, ref, pb.A) <= 4 * TOL["f64"], f"matrix {i} {pb.m}x{pb.n}"
            srv.close(mid)
        st = srv.stats()
        assert st["sweeps_done"] == len(tickets) and st["sweeps_failed"] == 0
        assert st["p99_us"] >= st["p50_us"] > 0
    assert rs.device_status(reset=True) == 0


def test_server_admission_under_budget():
    """Budget for two 256x256 matrices: four are opened; the later two wait
    for the first two to close, then complete; residency never exceeds it."""
    say("server: admission under a 2-matrix budget")
    m = n = 256
    one = m * n * 8
    pbs = [make_problem(m, n, 1, seed=70 + i) for i in range(4)]
    plans = [sweeps_for(i, n, 2, seed=1) for i in range(4)]
    with rs.Server(budget_bytes=2 * one) as srv:
        with pytest.raises(rs.RotseqError) as e:
            srv.open(np.zeros((512, 512)))
        assert e.value.code == 6  # ROTSEQ_E_BUDGET
        ids = [srv.open(pb.A) for pb in pbs]
        tickets = [[srv.submit(mid, C, S) for C, S in plans[i]] for i, mid in enumerate(ids)]
        for t in tickets[0] + tickets[1]:
            assert srv.wait(t)[0] == 0
        st = srv.stats()
        assert st["matrices_pending"] == 2 and st["resident_bytes"] <= 2 * one
        # the pending ones cannot run yet
        assert srv.wait(tickets[2][0], timeout_us=20000)[0] == 5  # ROTSEQ_E_TIMEOUT
        got01 = [srv.read(ids[i], m, n) for i in (0, 1)]
        srv.close(ids[0])
        srv.close(ids[1])
        for t in tickets[2] + tickets[3]:
            assert srv.wait(t)[0] == 0
        got23 = [srv.read(ids[i], m, n) for i in (2, 3)]
        for i, got in zip((0, 1, 2, 3), got01 + got23):
            assert relerr(got, oracle_sweeps(pbs[i].A, plans[i]), pbs[i].A) <= 2 * TOL["f64"]
        assert srv.stats()["peak_resident_bytes"] <= 2 * one
        for code, call in ((8, lambda: srv.submit(ids[0], *plans[0][0])),
                           (8, lambda: srv.read(ids[0], m, n)),
                           (7, lambda: srv.close(12345))):
            with pytest.raises(rs.RotseqError) as e:
                call()
            assert e.value.code == code
        assert srv.wait(987654)[0] == 7  # ROTSEQ_E_INVAL


def test_server_alone_equals_amid_traffic():
    """Batching with other matrices does not change a matrix's arithmetic."""
    say("server: alone vs amid traffic")
    pb = make_problem(300, 257, 1, seed=91)
    plan = sweeps_for(3, pb.n, 5, seed=2)
    with rs.Server() as srv:
        mid = srv.open(pb.A)
        ts = [srv.submit(mid, C, S) for C, S in plan]
        for t in ts:
            assert srv.wait(t)[0] == 0
        alone = srv.read(mid, pb.m, pb.n)
    others = [make_problem(m, n, 1, seed=200 + i) for i, (m, n) in enumerate(SHAPES * 3)]
    with rs.Server(max_batch=16) as srv:
        oids = [srv.open(o.A) for o in others]
        mid = srv.open(pb.A)
        ts = []
        for s, (C, S) in enumerate(plan):
            for j, oid in enumerate(oids):
                Co, So = sweeps_for(j, others[j].n, 1, seed=10 + s)[0]
                srv.submit(oid, Co, So)
            ts.append(srv.submit(mid, C, S))
        for t in ts:
            assert srv.wait(t)[0] == 0
        amid = srv.read(mid, pb.m, pb.n)
        assert srv.stats()["mean_batch"] > 1.0
    assert np.array_equal(alone, amid)
    assert relerr(alone, oracle_sweeps(pb.A, plan), pb.A) <= 5 * TOL["f64"]


def test_served_scale_requests_sampled_rows():
    """Requests of the served configuration at its own scale: n log-uniform
    in [128, 4096] (the largest drawn ones plus n = 4096 itself), k per
    request in {16, 32, 64, 128}, 20 sweeps each with fresh angles, all
    resident at once and batched together.  Every row's norm is kept, and
    sampled rows match the oracle applied sweep by sweep (rows are
    independent, so the oracle runs on those rows alone)."""
    from paper_2412_01852_amd.inputs import request_matrix, served_requests
    reqs = served_requests(48, seed=5)
    reqs = sorted(reqs, key=lambda r: -r["n"])[:3] + reqs[-3:]
    reqs.append(dict(reqs[0], m=4096, n=4096, k=128))
    say("server at served scale: " + ", ".join(f"n={r['n']} k={r['k']}" for r in reqs))
    work = []
    for r in reqs:
        A, rng = request_matrix(r)
        sweeps = [make_cs(r["n"], r["k"], rng) for _ in range(r["sweeps"])]
        work.append((A, sweeps))
    with rs.Server() as srv:
        ids = [srv.open(A) for A, _ in work]
        tickets = []
        for s in range(20):
            for mid, (_, sweeps) in zip(ids, work):
                tickets.append(srv.submit(mid, *sweeps[s]))
        for t in tickets:
            assert srv.wait(t)[0] == 0
        got = [srv.read(mid, A.shape[0], A.shape[1]) for mid, (A, _) in zip(ids, work)]
        st = srv.stats()
        assert st["sweeps_done"] == 20 * len(reqs) and st["sweeps_failed"] == 0
        assert st["mean_batch"] > 1.0
    assert rs.device_status(reset=True) == 0
    rng = np.random.default_rng(7)
    for (A, sweeps), g, r in zip(work, got, reqs):
        m = A.shape[0]
        rows = np.unique(np.concatenate([[0, 63, 64, m - 1], rng.choice(m, 12, replace=False)]))
        ref = oracle_sweeps(A[rows], sweeps)
        err = relerr(g[rows], ref, A[rows])
        drift = np.max(np.abs(np.linalg.norm(g, axis=1) / np.linalg.norm(A, axis=1) - 1.0))
        say(f"  n={r['n']} k={r['k']}: rel err {err:.3e}, row-norm drift {drift:.1e}")
        assert err <= 4 * TOL["f64"], (r["n"], r["k"])
        assert drift <= 1e-12
