"""CPU model of the chain kernel's LDS hand-off protocol.

A producer wave writes columns into a ring of RB slots and a consumer wave
reads them, both in groups of G columns.  Each side publishes its counter
(produced / consumed) after every column (the kernel's LDS atomic add; the
older protocol published at the end of a group, still modelled), and polls
its neighbour's counter at the last step of a group for use at the start of
the next one (or, in the older protocol, at the start of the previous group).
At the start of a group a side checks whether the group is allowed; if not,
it waits until its neighbour's counter reaches the group's need plus extra
headroom (IN_SLACK columns for the consumer, OUT_SLACK slots for the
producer), exactly as the kernel does.

The model runs both sides with random relative speeds and checks that the
pair always finishes (no deadlock), that no column is read before it was
written and that no slot is overwritten before it was read.  With the
kernel's constants (RB = 16, G = 4, slack bound RB + 1 - 2G) it must always
finish; with too much slack it must find a deadlock, which shows the model
can see one.
"""
import random

import pytest

RB, G = 16, 4
SLACK = RB + 1 - 2 * G   # the deadlock-free bound on IN_SLACK + OUT_SLACK
IN_SLACK = OUT_SLACK = 0  # what the kernel asks for


def simulate(n, k_lag, d_cons, in_slack, out_slack, seed, max_ticks=400000, per_step=True):
    """True if producer and consumer both finish, False on deadlock.

    per_step: counters published after every column and polled at the last
    step of the previous group (the kernel); False: published at group ends
    and polled at the start of the previous group.

    Producer step t outputs column t - k_lag + 1; consumer step t fetches
    column t + d_cons + 1 after a preload of columns 0..d_cons.  Columns
    outside [0, n) move without waiting, as in the kernel.
    """
    rng = random.Random(seed)
    total = n + k_lag + 40
    produced = consumed = 0
    slot = {}  # slot -> column held
    # producer
    p_t, sc, p_wait = 0, -(k_lag - 1), None
    p_poll = 0   # consumed, as read at the producer's previous group start
    p_known = 0  # largest consumed value the producer has seen
    # consumer
    c_t, lc, c_wait, preloaded = 0, 0, None, False
    c_poll = 0   # produced, as read at the consumer's previous group start
    c_known = 0  # largest produced value the consumer has seen

    for _ in range(max_ticks):
        if p_t >= total and c_t >= total:
            return True
        moved = False
        # --- consumer
        if c_wait is not None and produced >= c_wait:
            c_wait = None
            c_known = produced
        if c_wait is None and c_t < total and rng.random() < 0.5:
            if not preloaded:
                need = min(d_cons + 1, n)
                if produced >= need:
                    for c in range(min(d_cons + 1, n)):
                        assert slot.get(c % RB) == c, "read before write"
                    lc = d_cons + 1
                    consumed = lc
                    preloaded = True
                    moved = True
                else:
                    c_wait = min(d_cons + 1 + in_slack, n)
            else:
                if c_t % G == 0 and c_wait is None:
                    c_known = max(c_known, c_poll)
                    if not per_step:
                        c_poll = produced
                if per_step and c_t % G == G - 1:
                    c_poll = produced
                if c_t % G == 0 and lc < n and c_known < min(lc + G, n):
                    c_wait = min(lc + G + in_slack, n)
                else:
                    if lc < n:
                        assert slot.get(lc % RB) == lc, "read before write"
                    lc += 1
                    c_t += 1
                    if per_step or c_t % G == 0:
                        consumed = lc
                    moved = True
        # --- producer
        if p_wait is not None and consumed >= p_wait:
            p_wait = None
            p_known = consumed
        if p_wait is None and p_t < total and rng.random() < 0.5:
            if p_t % G == 0:
                p_known = max(p_known, p_poll)
                if not per_step:
                    p_poll = consumed
            if per_step and p_t % G == G - 1:
                p_poll = consumed
            if p_t % G == 0 and sc + G > p_known + RB:
                p_wait = sc + G - RB + out_slack
            else:
                if 0 <= sc:
                    old = slot.get(sc % RB)
                    assert old is None or old >= n or old < consumed, "overwrote unread slot"
                    slot[sc % RB] = sc
                sc += 1
                p_t += 1
                if per_step or p_t % G == 0:
                    produced = sc
                moved = True
        c_stuck = c_wait is not None and produced < c_wait
        p_stuck = p_wait is not None and consumed < p_wait
        if c_stuck and (p_stuck or p_t >= total):
            return False  # the consumer can never be satisfied
        if p_stuck and c_t >= total:
            return False  # the producer can never be satisfied
    return False


@pytest.mark.parametrize("per_step", [True, False])
@pytest.mark.parametrize("seed", range(30))
@pytest.mark.parametrize("k_lag,d_cons", [(6, 1), (4, 3), (8, 7), (6, 9)])
@pytest.mark.parametrize("n", [5, 37, 300])
def test_protocol_finishes(seed, k_lag, d_cons, n, per_step):
    assert simulate(n, k_lag, d_cons, IN_SLACK, OUT_SLACK, seed, per_step=per_step)


@pytest.mark.parametrize("per_step", [True, False])
def test_model_detects_deadlock_with_too_much_slack(per_step):
    """Slack 8 + 7 with G = 4 (above the bound) deadlocks once a side decides
    to wait on a stale counter: the model must find it."""
    results = [simulate(300, 8, 7, 8, 7, seed, per_step=per_step) for seed in range(60)]
    assert not all(results)


def test_bound_is_tight_for_per_step_protocol():
    """One slot of slack above RB + 1 - 2G (6 + 4) already deadlocks."""
    assert 6 + 4 == RB + 2 - 2 * G
    results = [simulate(300, 8, 7, 6, 4, seed) for seed in range(60)]
    assert not all(results)


def test_slack_bound():
    assert IN_SLACK + OUT_SLACK <= RB + 1 - 2 * G
    assert IN_SLACK >= 0 and OUT_SLACK >= 0


@pytest.mark.parametrize("per_step", [True, False])
@pytest.mark.parametrize("seed", range(20))
def test_protocol_finishes_at_the_bound(seed, per_step):
    """Headroom exactly at the bound (5 + 4) is still deadlock-free."""
    for k_lag, d_cons in [(6, 1), (8, 7), (4, 3)]:
        assert simulate(300, k_lag, d_cons, 5, 4, seed, per_step=per_step)
