"""Pins of the oracle's change detection (Sec. III.B: the moving window set against the
Accumulator to detect an attack or a need to reprocess; the measure is our reading: an alarm
when some value's share of the window differs from its share of the Accumulator by more than
alarm_pct percentage points, strict).

The expected values below are worked out by hand from that definition (shares of small
streams, closed forms), not by calling the oracle's formula again; invariants that any share
comparison must satisfy cover the rest, and planted mistakes show that the pins notice the
plausible errors (the Accumulator taken before the window, a dropped absolute value, a
non-strict test)."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O


def u8(values):
    return np.array(values, dtype=np.uint8)


def alarms(chunks, W, alarm_pct, lag=0):
    return O.stream_reference(chunks, W=W, theta_pct=45, S=960, rmax=8, lag=lag, alarm_pct=alarm_pct)["alarms"]


def test_hand_example_new_value_takes_the_window():
    # three chunks 0,1,2,3 then one chunk 7,7,7,7; W = 1.  After the last chunk the window is
    # all 7 (share 1) while the Accumulator holds 4 sevens in 16 bytes (share 1/4): 3/4 apart.
    chunks = [u8([0, 1, 2, 3])] * 3 + [u8([7, 7, 7, 7])]
    assert O.share_departure(O.hist(chunks[3]), [3, 3, 3, 3, 0, 0, 0, 4] + [0] * 248) == Fraction(3, 4)
    assert alarms(chunks, 1, 74) == [0, 0, 0, 1]
    assert alarms(chunks, 1, 75) == [0, 0, 0, 0]      # exactly 75 points apart: not more
    assert alarms(chunks, 1, 1) == [0, 0, 0, 1]       # the first three chunks agree exactly


def test_hand_example_value_vanishes():
    # eight 5s then eight 6s, W = 1: value 5 falls from 1/2 of the Accumulator to 0 of the
    # window, value 6 rises from 1/2 to 1: 1/2 apart either way
    chunks = [u8([5] * 8), u8([6] * 8)]
    assert alarms(chunks, 1, 49) == [0, 1]
    assert alarms(chunks, 1, 50) == [0, 0]


def test_closed_form_uniform_then_constant():
    # n chunks holding every value c times, then m chunks of c * 256 copies of v, W = m:
    # the window is all v; the Accumulator's share of v is (n c + m 256 c) / ((n + m) 256 c)
    for n, m, c, v in [(3, 1, 1, 9), (5, 2, 3, 200), (1, 4, 2, 0), (17, 3, 1, 255)]:
        chunks = [u8(np.repeat(np.arange(256), c))] * n + [u8([v] * (256 * c))] * m
        dep = 1 - Fraction(n + 256 * m, 256 * (n + m))
        pct = dep * 100
        below = int(pct) - (1 if pct == int(pct) else 0)       # largest integer < pct
        assert alarms(chunks, m, below)[-1] == 1, (n, m, c, v)
        assert alarms(chunks, m, int(pct) + 1 if pct != int(pct) else int(pct))[-1] == 0, (n, m, c, v)
        # the chunks before the change never alarm: their windows share the Accumulator's shape
        assert alarms(chunks, m, 1)[:n] == [0] * n


def test_window_covering_the_stream_never_alarms():
    g = np.random.default_rng(7)
    chunks = [u8(g.integers(0, 256, int(g.integers(1, 500)))) for _ in range(12)]
    # for k < W the window is the Accumulator
    assert alarms(chunks, 12, 1) == [0] * 12
    assert alarms(chunks, 64, 1) == [0] * 12


def test_stationary_stream_never_alarms():
    # every chunk a permutation of the same bytes: every window has the Accumulator's shares
    g = np.random.default_rng(11)
    base = g.integers(0, 256, 4096).astype(np.uint8)
    chunks = [g.permutation(base) for _ in range(20)]
    for W in (1, 3, 8):
        assert alarms(chunks, W, 1) == [0] * 20


def test_empty_histograms_never_alarm():
    chunks = [u8([]), u8([]), u8([4, 4]), u8([])]
    # after chunk 3 (W = 1) the window is empty; before chunk 2 the Accumulator is
    assert alarms(chunks, 1, 1) == [0, 0, 0, 0]
    assert O.share_departure([0] * 256, [1] + [0] * 255) == 0
    assert O.share_departure([1] + [0] * 255, [0] * 256) == 0


def test_alarm_off_at_zero():
    chunks = [u8([0] * 10), u8([1] * 10)]
    assert alarms(chunks, 1, 0) == [0, 0]


def test_invariant_under_value_relabelling_and_scaling():
    g = np.random.default_rng(3)
    chunks = []
    for k in range(16):
        if k in (6, 7, 12):
            chunks.append(u8([int(g.integers(0, 256))] * 700))
        else:
            chunks.append(g.integers(0, 256, 700).astype(np.uint8))
    perm = g.permutation(256).astype(np.uint8)
    for W, pct in [(1, 20), (2, 10), (4, 5)]:
        ref = alarms(chunks, W, pct)
        assert sum(ref) > 0
        assert alarms([perm[c] for c in chunks], W, pct) == ref                 # relabel the values
        assert alarms([np.concatenate([c, c]) for c in chunks], W, pct) == ref  # every count doubled
        assert alarms(chunks, W, pct, lag=3) == ref                             # lag moves decisions only


def test_alarm_is_monotone_in_the_threshold():
    g = np.random.default_rng(5)
    chunks = [g.integers(0, 256, 300).astype(np.uint8) if k % 5 else u8([k] * 300) for k in range(30)]
    prev = None
    for pct in range(0, 101, 5):
        a = alarms(chunks, 3, pct) if pct else [1] * 30
        if prev is not None:
            assert all(x <= y for x, y in zip(a, prev))
        prev = a
    assert alarms(chunks, 3, 100) == [0] * 30    # shares differ by at most 1


def test_planted_mistakes_are_caught():
    # Three plausible mistakes; each must fail one of the pins above.
    def acc_before_window(mw, acc, pct):      # Accumulator without the window's chunks
        rest = [a - m for a, m in zip(acc, mw)]
        return O.change_alarm(mw, rest, pct)

    def no_abs(mw, acc, pct):                 # only rises of a share are seen
        n1, n2 = sum(mw), sum(acc)
        if not n1 or not n2 or not pct:
            return False
        return max(Fraction(m, n1) - Fraction(a, n2) for m, a in zip(mw, acc)) > Fraction(pct, 100)

    def not_strict(mw, acc, pct):
        return bool(pct) and O.share_departure(mw, acc) >= Fraction(pct, 100)

    seven = [3, 3, 3, 3, 0, 0, 0, 4] + [0] * 248          # the Accumulator of the first example
    mw7 = [0] * 7 + [4] + [0] * 248
    # the Accumulator taken before the window puts 7 at share 0: 100 points, alarm at 75
    assert acc_before_window(mw7, seven, 75) and not O.change_alarm(mw7, seven, 75)
    # a value that vanishes from the window only lowers shares... except the one that rises;
    # a value that vanishes while the rest keep their shares is missed without the absolute
    acc = [8, 8] + [0] * 254
    mw = [0, 8] + [0] * 254
    assert O.change_alarm(mw, acc, 49)
    acc3 = [10, 10, 10, 10] + [0] * 252       # four values, one vanishes from the window
    mw3 = [0, 10, 10, 10] + [0] * 252
    assert O.change_alarm(mw3, acc3, 8) and not no_abs(mw3, acc3, 9)
    assert O.share_departure(mw3, acc3) == Fraction(1, 4)
    # exactly on the threshold
    assert not_strict(mw7, seven, 75) and not O.change_alarm(mw7, seven, 75)
