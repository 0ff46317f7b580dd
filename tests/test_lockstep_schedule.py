"""CPU model of the chain kernel's lockstep schedule inside a workgroup.

The waves of a workgroup advance in groups of G steps that all end at one
workgroup barrier, after each wave's LDS accesses of the group have
completed.  A wave at position p of its chain segment spends LG*p idle
groups, one prologue group (fetching its first D+1 input columns), steps/G
groups of steps (step s in group LG*p + 1 + s // G), and idle groups up to a
common count.  Its LDS output ring has RB slots; the wave writes column c
(the output of its step c + K - 1) into slot c mod RB.

A group orders everything before its barrier before everything after it,
and nothing inside it, so hand-off through a slot is safe exactly when, for
every column c, the producer's write group < the consumer's read group <
the group of the producer's next write to the same slot.  The test checks
that with the kernel's constants for every band width, that one group less
of lag breaks it (so the lag is the smallest), and that every wave of every
workgroup passes the same number of barriers whatever its position and
segment offset, which keeps the barriers matched.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHAIN = os.path.join(ROOT, "paper_2412_01852_amd", "csrc", "rotseq_chain.hip")

U, RB, G = 16, 16, 4


def geometry(K):
    r_lds = 8 if K <= 6 else 16
    return r_lds - K - 1  # D of an LDS-fed wave


def kernel_lag(K):
    """LG as the kernel source defines it."""
    src = open(CHAIN).read()
    m = re.search(r"static constexpr int LG = K == 8 \? (\d+) : (\d+);", src)
    assert m, "LG definition not found in the chain kernel"
    return int(m.group(1)) if K == 8 else int(m.group(2))


def kernel_constants():
    src = open(CHAIN).read()
    get = lambda name: int(re.search(r"static constexpr int %s = (\d+);" % name, src).group(1))  # noqa: E731
    return get("U"), get("RB"), get("G")


def violations(K, lg, steps, G=G, RB=RB):
    """Columns whose slot hand-off is unsafe under lag `lg` (producer at
    position 0, consumer at position 1), with groups of G steps and RB-slot
    channels."""
    D = geometry(K)
    write = lambda c: 1 + (c + K - 1) // G  # noqa: E731  producer group writing column c

    def read(c):  # consumer group reading column c
        return lg if c <= D else lg + 1 + (c - 1 - D) // G

    last_out = steps - K  # last column the producer writes (its step steps-1)
    bad = []
    for c in range(0, steps + D + 1):  # every column the consumer reads
        if c <= last_out and not write(c) < read(c):
            bad.append(("read before write", c))
        if c + RB <= last_out and not read(c) < write(c + RB):
            bad.append(("overwritten before read", c))
    return bad


def test_constants_match_kernel():
    assert kernel_constants() == (U, RB, G)


# The streaming form (whole chains per workgroup): longer groups, larger
# channels, its own lag.
def deep_constants():
    src = open(CHAIN).read()
    get = lambda name: int(re.search(r"static constexpr int %s = (\d+);" % name, src).group(1))  # noqa: E731
    m = re.search(r"static constexpr int LG_deep = K == 8 \? (\d+) : (\d+);", src)
    assert m, "LG_deep definition not found in the chain kernel"
    return get("G_deep"), get("RB_deep"), get("H_deep"), (int(m.group(1)), int(m.group(2)))


@pytest.mark.parametrize("K", [2, 4, 6, 8])
@pytest.mark.parametrize("steps", [32, 64, 4128])
def test_streaming_lag_is_safe_and_smallest(K, steps):
    g, rb, h, (lg8, lg) = deep_constants()
    lag = lg8 if K == 8 else lg
    assert (U * h) % rb == 0 and U % g == 0
    assert violations(K, lag, steps, g, rb) == []
    if steps > 64:
        assert violations(K, lag - 1, steps, g, rb), "a smaller lag would do"


@pytest.mark.parametrize("K", [2, 4, 6, 8])
@pytest.mark.parametrize("steps", [16, 32, 10256])
def test_kernel_lag_is_safe(K, steps):
    assert violations(K, kernel_lag(K), steps) == []


@pytest.mark.parametrize("K", [2, 4, 6, 8])
def test_kernel_lag_is_smallest(K):
    assert violations(K, kernel_lag(K) - 1, 10256), "a smaller lag would do"


@pytest.mark.parametrize("K", [2, 4, 6, 8])
def test_too_much_lag_overwrites(K):
    """The ring bounds the lag from above too: the model sees overwrites."""
    assert any(kind == "overwritten before read"
               for kind, _ in violations(K, kernel_lag(K) + RB // G, 10256))


def kernel_dg():
    src = open(CHAIN).read()
    return int(re.search(r"static constexpr int DG = (\d+);", src).group(1))


def segment_offset(b0, W, lg, dg):
    """The kernel's closed form (segment_offset in the chain kernel)."""
    if b0 <= 0:
        return 0
    r = (b0 - 1) % W + 1
    q = (b0 - r) // W
    return q * (lg * (W - 1) + dg) + lg * (r - 1) + dg


def segment_offset_recursive(b0, W, lg, dg):
    """The definition: a segment starting at band b0 > 0 follows the last
    wave of the previous workgroup, at position min(W, b0) - 1 of a segment
    starting at band b0 - min(W, b0), by DG groups."""
    if b0 == 0:
        return 0
    r = min(W, b0)
    return segment_offset_recursive(b0 - r, W, lg, dg) + lg * (r - 1) + dg


@pytest.mark.parametrize("W", [1, 2, 3, 8, 15, 16])
def test_segment_offset_closed_form(W):
    lg, dg = kernel_lag(8), kernel_dg()
    for b0 in range(0, 200):
        assert segment_offset(b0, W, lg, dg) == segment_offset_recursive(b0, W, lg, dg)


def workgroup_barriers(g, W, tiles, nbands, steps, lg, dg):
    """Barriers each wave of workgroup g passes, following chain_workgroup
    and bandwave: pre idle groups, the prologue group, steps/G groups, post
    idle groups; idle waves pass max_pre + 1 + steps/G."""
    total = tiles * nbands
    pres = []
    for v in range(W):
        iv = g * W + v
        if iv >= total:
            break
        bv = iv % nbands
        pv = min(v, bv)
        pres.append(segment_offset(bv - pv, W, lg, dg) + lg * pv)
    max_pre = max(pres) if pres else 0
    counts = []
    for w in range(W):
        if g * W + w >= total:
            counts.append(max_pre + 1 + steps // G)
        else:
            pre = pres[w]
            counts.append(pre + 1 + steps // G + (max_pre - pre))
    return counts


@pytest.mark.parametrize("K", [2, 4, 6, 8])
@pytest.mark.parametrize("W,tiles,nbands", [(1, 3, 5), (2, 5, 3), (8, 7, 24), (16, 160, 24),
                                           (16, 3, 5), (15, 11, 40), (16, 2, 100)])
def test_every_wave_passes_the_same_barriers(K, W, tiles, nbands):
    """Every wave of every workgroup (idle waves of the last one included)
    passes the same number of barriers."""
    lg, dg, steps = kernel_lag(K), kernel_dg(), 10256 // U * U
    nwg = -(-tiles * nbands // W)
    for g in range(nwg):
        counts = workgroup_barriers(g, W, tiles, nbands, steps, lg, dg)
        assert len(set(counts)) == 1, (g, counts)


def test_offsets_keep_neighbours_in_a_segment_lg_apart():
    """Within a segment the lag between neighbours stays LG (the LDS
    hand-off condition); segments only move as a whole."""
    lg, dg, W, nbands = kernel_lag(8), kernel_dg(), 16, 24
    for g in range(30):
        prev = None
        for v in range(W):
            iv = g * W + v
            bv, tile = iv % nbands, iv // nbands
            pv = min(v, bv)
            pre = segment_offset(bv - pv, W, lg, dg) + lg * pv
            if prev is not None and prev[0] == tile and pv > 0:
                assert pre - prev[1] == lg
            prev = (tile, pre)
