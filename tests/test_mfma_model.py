"""CPU checks of the matrix-instruction sweep's window decomposition and
schedule (models in tests/mfma_model.py): the windowed application equals
the oracle; every window matrix is orthogonal with the band structure the
kernel relies on; every ring slot and published block is produced before
it is used and not overwritten before it is read."""
import numpy as np
import pytest

import oracle
from mfma_model import (FLAG_MARGIN, KB, POLL_LAG, band_model, block_cols, nwin_of, qsw_layout, schedule_events,
                        seg_delay, sweep_model, total_steps, wave_stride, window_q)
from paper_2412_01852_amd.inputs import make_problem


@pytest.mark.parametrize("m,n,k", [(5, 2, 1), (3, 3, 9), (7, 9, 8), (4, 17, 13), (6, 40, 24),
                                   (2, 33, 3), (9, 16, 16), (3, 8, 40)])
def test_windowed_sweep_equals_oracle(m, n, k):
    pb = make_problem(m, n, k, seed=100 + 7 * n + k)
    ref = oracle.colmajor(np.asarray(pb.A))
    oracle.rotseq(ref, oracle.colmajor(pb.C), oracle.colmajor(pb.S))
    got = sweep_model(np.asarray(pb.A), np.asarray(pb.C), np.asarray(pb.S))
    err = np.linalg.norm(got - np.asarray(ref)) / np.linalg.norm(np.asarray(pb.A))
    assert err <= 1e-14, err


def test_window_matrices_orthogonal_and_banded():
    """Q(band, w) is orthogonal, and Q[i, c] = 0 for i > c + 8: a band of 8
    sequences moves an input column at most 8 places to the left.  Window
    -1 leaves the virtual columns -8..-1 (rows and columns 0..7 of Q) alone,
    and a window past the last column is the identity."""
    pb = make_problem(1, 50, 20, seed=5)
    C, S = np.asarray(pb.C), np.asarray(pb.S)
    for band in range(3):
        for w in range(-1, nwin_of(50)):
            Q = window_q(C, S, 50, 20, band, w)
            assert np.allclose(Q.T @ Q, np.eye(16), atol=1e-14)
            i, c = np.indices(Q.shape)
            assert np.all(Q[i > c + KB] == 0.0)
        Qm = window_q(C, S, 50, 20, band, -1)
        assert np.array_equal(Qm[:KB, :], np.eye(16)[:KB, :])
        assert np.array_equal(Qm[:, :KB], np.eye(16)[:, :KB])
    assert np.array_equal(window_q(C, S, 50, 20, 0, nwin_of(50) + 1), np.eye(16))


def test_blocks_cover_every_column_once():
    for n in (2, 3, 8, 9, 15, 16, 17, 100):
        cols = np.concatenate([block_cols(v) for v in range(nwin_of(n))])
        real = cols[(cols >= 0) & (cols < n)]
        assert np.array_equal(np.sort(real), np.arange(n))
        # the block after the last window holds only virtual columns
        assert block_cols(nwin_of(n))[0] >= n
        # the last window ends at or after the band's last step, n + 5
        assert KB * (nwin_of(n) - 1) + 2 * KB - 2 >= n + 5


def test_single_band_mutant_caught():
    """A window skipped (or applied twice) must break the equality."""
    pb = make_problem(4, 30, 8, seed=9)
    A, C, S = np.asarray(pb.A), np.asarray(pb.C), np.asarray(pb.S)
    good = band_model(A, C, S, 0)
    ref = oracle.colmajor(A.copy())
    oracle.rotseq(ref, oracle.colmajor(C), oracle.colmajor(S))
    assert np.allclose(good, np.asarray(ref), atol=1e-13)
    C2 = C.copy()
    C2[11, 3], S[11, 3] = 1.0, 0.0  # drop one rotation
    bad = band_model(A, C2, S, 0)
    assert not np.allclose(bad, np.asarray(ref), atol=1e-6)


def test_qsw_layout_matches_matrix_operand():
    """Lane l, slab s of the stored window holds Q[4s + l//16, l%16] (the
    A operand of v_mfma_f64_16x16x4f64 for Q^T: row = l%16, k = l//16)."""
    Q = np.arange(256, dtype=np.float64).reshape(16, 16)
    L = qsw_layout(Q)
    for lane in (0, 15, 16, 37, 63):
        for s in range(4):
            assert L[lane, s] == Q[4 * s + lane // 16, lane % 16]


@pytest.mark.parametrize("nb_wave", [1, 2, 3])
@pytest.mark.parametrize("active", [1, 2, 3, 4])
@pytest.mark.parametrize("nwin", [1, 2, 5, 17])
def test_schedule_dependencies(nb_wave, active, nwin):
    """Within a workgroup: band i consumes band i-1's block of the previous
    super-step (so the bands of a super-step are independent); every ring,
    stage and store slot is written in a strictly earlier super-step than
    it is read and not rewritten (4 slots) until after that read; loads are
    two super-steps old when staged; every event lies inside the
    workgroup's super-steps."""
    ev = schedule_events(nb_wave, nwin, active=active)
    T = total_steps(nb_wave, nwin)
    mf = {(e[1], e[2], e[3]): e[4] for e in ev if e[0] == "mfma"}
    for (j, i, w), t in mf.items():
        if i > 0 and w + 1 <= nwin - 1:
            assert mf[(j, i - 1, w + 1)] == t - 1
    ring_w = {(e[1], e[2]): e[4] for e in ev if e[0] == "ring_w"}
    for e in ev:
        if e[0] == "ring_r":
            _, j, v, slot, t = e
            assert ring_w[(j - 1, v)] < t
            assert ring_w.get((j - 1, v + 4), T) > t
            assert mf[(j, 0, v - 1)] == t  # band 0 takes block v at window v-1
    load = {e[1]: e[2] for e in ev if e[0] == "load"}
    stage_w = {e[1]: e[3] for e in ev if e[0] == "stage_w"}
    for e in ev:
        if e[0] == "stage_r":
            _, v, slot, t = e
            assert load[v] + 2 <= stage_w[v] < t
            assert stage_w.get(v + 4, T) > t
            assert mf[(0, 0, v - 1)] == t
    out = active - 1
    for e in ev:
        if e[0] == "store":
            _, v, slot, t = e
            assert ring_w[(out, v)] < t < ring_w[(out, v + 4)] if (out, v + 4) in ring_w else ring_w[(out, v)] < t
    for e in ev:
        if e[0] in ("mfma", "ring_w", "ring_r", "stage_r", "store"):
            assert 0 <= e[-1] < T, e
        if e[0] in ("load", "stage_w"):
            assert e[-1] < T, e  # loads before the segment's start fetch empty blocks


@pytest.mark.parametrize("nb_wave", [1, 2, 3])
def test_segment_handoff_margin(nb_wave):
    """The waves of segment s+1 load block v at their super-step v-3 using
    a flag poll issued POLL_LAG super-steps earlier; segment s publishes v
    at least FLAG_MARGIN super-steps before that poll."""
    nwin = 20
    for seg in (1, 2):
        pub = {e[1]: e[2] for e in schedule_events(nb_wave, nwin, seg - 1) if e[0] == "publish"}
        load = {e[1]: e[2] for e in schedule_events(nb_wave, nwin, seg) if e[0] == "load"}
        for v in range(0, nwin):
            assert load[v] - POLL_LAG >= pub[v] + FLAG_MARGIN, (seg, v)
    assert seg_delay(nb_wave) % 4 == 0 and wave_stride(nb_wave) % 4 == 0
