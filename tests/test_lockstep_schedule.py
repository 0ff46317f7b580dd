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
of lag breaks it (so the lag is the smallest), and that every wave passes
the same number of barriers whatever its position, which is what keeps the
barrier from deadlocking.
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


def violations(K, lg, steps):
    """Columns whose slot hand-off is unsafe under lag `lg` (producer at
    position 0, consumer at position 1)."""
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


@pytest.mark.parametrize("K", [4, 6, 8])
@pytest.mark.parametrize("steps", [16, 32, 10256])
def test_kernel_lag_is_safe(K, steps):
    assert violations(K, kernel_lag(K), steps) == []


@pytest.mark.parametrize("K", [4, 6, 8])
def test_kernel_lag_is_smallest(K):
    assert violations(K, kernel_lag(K) - 1, 10256), "a smaller lag would do"


@pytest.mark.parametrize("K", [4, 6, 8])
def test_too_much_lag_overwrites(K):
    """The ring bounds the lag from above too: the model sees overwrites."""
    assert any(kind == "overwritten before read"
               for kind, _ in violations(K, kernel_lag(K) + RB // G, 10256))


@pytest.mark.parametrize("K", [4, 6, 8])
@pytest.mark.parametrize("waves", [1, 2, 8, 16])
def test_every_wave_passes_the_same_barriers(K, waves):
    """Barrier count per wave as the kernel runs it: idle waves and every
    position in a segment end up at LG*(W-1) + 1 + steps/G."""
    lg, steps = kernel_lag(K), 10256 // U * U
    idle = lg * (waves - 1) + 1 + steps // G
    for pos in range(waves):
        active = lg * pos + 1 + steps // G + lg * (waves - 1 - pos)
        assert active == idle
