"""CPU model of the 3x3 reflector sweep's lockstep schedule.

The constants of R3Geom are read from the kernel source.  The model replays
what every wave of a workgroup does, group by group (wave w idles for
w*L/G groups, fetches its first D+2 columns, then runs its steps; every G
steps end a group): it checks that every column a wave takes from its
neighbour's LDS ring was written in an earlier group and not overwritten
before the reading group, that no slot is written and read by different
waves in one group, that every wave passes the same number of barriers, and
it carries the arithmetic through the schedule to compare with the oracle.
"""
import os
import re

import numpy as np
import pytest

import oracle
from oracle_pins import colmajor, relerr

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2412_01852_amd", "csrc", "rotseq_refl3.hip")


def geometry(K):
    with open(SRC) as f:
        src = f.read()
    body = src[src.index("struct R3Geom {"):]
    body = body[:body.index("};")]
    env = {"K": K}
    for name in ("G", "D", "R", "L", "RB"):
        expr = re.search(rf"static constexpr int {name} = ([^;]+);", body).group(1)
        env[name] = eval(expr.replace("/", "//"), {}, dict(env))
    return env


def band_plan(n, K, R):
    steps = n + 2 * K - 2
    return (steps + R - 1) // R * R


def simulate(m, n, k, K, W, A=None, coef=None, check=True):
    """Replays one launch of W waves (bands 0..W-1, sequences 0..k-1) on the
    rows of A (m x n, modified in place when given).  Returns the number of
    barriers each wave passed."""
    g = geometry(K)
    G, D, R, L, RB = g["G"], g["D"], g["R"], g["L"], g["RB"]
    steps = band_plan(n, K, R)
    chunks = steps // R
    kq_last = min(K, k - (W - 1) * K)
    events = []  # (group, wave, op, ring, slot, column)
    barriers = [0] * W
    x = [[None] * R for _ in range(W)]
    rings = [[None] * RB for _ in range(W)]
    vals = A is not None

    def fetch(w, c, group):
        if c >= n:
            return np.zeros(m) if vals else None
        if w == 0:
            return A[:, c].copy() if vals else None
        events.append((group, w, "r", w - 1, c % RB, c))
        return rings[w - 1][c % RB]

    def put(w, c, v, group):
        if c < 0 or c >= n:
            return
        if w == W - 1:
            if vals:
                A[:, c] = v
        else:
            events.append((group, w, "w", w, c % RB, c))
            rings[w][c % RB] = v

    # The waves run concurrently; the model runs them one after the other
    # group by group (wave order reversed inside a group, so a missing
    # barrier would show as a stale value), which is valid when the event
    # check below finds no same-group conflicts.
    pre = [w * (L // G) for w in range(W)]
    total = pre[W - 1] + chunks * (R // G) + (W - 1) * (L // G) - pre[W - 1]
    state = [{"t": 0, "started": False} for _ in range(W)]
    for group in range(total):
        for w in reversed(range(W)):
            if group < pre[w] or group >= pre[w] + chunks * (R // G):
                barriers[w] += 1
                continue
            st = state[w]
            kq = kq_last if w == W - 1 else K
            if not st["started"]:
                st["started"] = True
                x[w] = [np.zeros(m) if vals else None for _ in range(R)]
                for c in range(D + 2):
                    x[w][c] = fetch(w, c, group)
            for _ in range(G):
                t = st["t"]
                u = t % R
                x[w][(u + 2 + D) % R] = fetch(w, t + 2 + D, group)
                for q in range(K):
                    j = t - 2 * q
                    if q >= kq or j < 0 or j >= n - 2:
                        continue
                    if vals:
                        p = w * K + q
                        tau, nu1, nu2 = coef[0][j, p], coef[1][j, p], coef[2][j, p]
                        s = (u - 2 * q) % R
                        xx, yy, zz = x[w][s], x[w][(s + 1) % R], x[w][(s + 2) % R]
                        wv = xx + nu1 * yy + nu2 * zz
                        tw = tau * wv
                        x[w][s], x[w][(s + 1) % R], x[w][(s + 2) % R] = xx - tw, yy - nu1 * tw, zz - nu2 * tw
                put(w, t - 2 * K + 2, x[w][(u - 2 * K + 2) % R], group)
                st["t"] += 1
            barriers[w] += 1
    if check:
        by_slot = {}
        for ev in events:
            by_slot.setdefault((ev[3], ev[4]), []).append(ev)
        for (ring, slot), evs in by_slot.items():
            writes = [e for e in evs if e[2] == "w"]
            for e in evs:
                if e[2] != "r":
                    continue
                group, _, _, _, _, c = e
                before = [wr for wr in writes if wr[0] < group]
                assert before and before[-1][5] == c, f"ring {ring} slot {slot}: column {c} read in group {group} not the last write"
                assert not any(wr[0] == group for wr in writes), f"ring {ring} slot {slot}: write and read in group {group}"
    return barriers


@pytest.mark.parametrize("K", [4, 8])
def test_geometry_conditions(K):
    g = geometry(K)
    G, D, R, L, RB = g["G"], g["D"], g["R"], g["L"], g["RB"]
    assert R >= 2 * K + 1 + D and R % G == 0
    assert L >= 2 * K + D + G and L % G == 0
    assert RB >= 2 * G - 1 and RB >= L + G - 2 * K + 2
    assert (12 - 1) * RB * 64 * 8 <= 160 * 1024, "FP64 rings of 12 waves must fit the LDS"


@pytest.mark.parametrize("K", [4, 8])
@pytest.mark.parametrize("n,k,W", [(3, 8, 1), (5, 16, 2), (40, 24, 3), (97, 40, 5), (131, 93, 12), (300, 96, 12)])
def test_lockstep_events(n, k, W, K):
    """No ring slot is read before its column was written, after it was
    overwritten, or in the group of a write; barrier counts are equal."""
    k = min(k, W * K)
    barriers = simulate(1, n, k, K, W)
    assert len(set(barriers)) == 1, barriers


@pytest.mark.parametrize("K", [4, 8])
@pytest.mark.parametrize("m,n,k", [(3, 3, 1), (5, 4, 9), (7, 23, 17), (2, 61, 40), (4, 150, 96)])
def test_schedule_matches_oracle(m, n, k, K):
    """The schedule (all launches of at most 12 waves) carries the arithmetic
    to the oracle's result within rounding."""
    rng = np.random.Generator(np.random.PCG64(1000 + n))
    nu1, nu2 = rng.standard_normal((n - 2, k)), rng.standard_normal((n - 2, k))
    tau = 2.0 / (1.0 + nu1 ** 2 + nu2 ** 2)
    A0 = rng.standard_normal((m, n))
    A = A0.copy()
    nb = (k + K - 1) // K
    launches = (nb + 11) // 12
    waves = (nb + launches - 1) // launches
    for b0 in range(0, nb, waves):
        W = min(waves, nb - b0)
        p0, p1 = b0 * K, min(k, (b0 + W) * K)
        simulate(m, n, p1 - p0, K, W, A, (tau[:, p0:p1], nu1[:, p0:p1], nu2[:, p0:p1]))
    ref = colmajor(A0)
    oracle.refl3seq(ref, colmajor(tau), colmajor(nu1), colmajor(nu2))
    assert relerr(A, np.asarray(ref)) <= 1e-13
