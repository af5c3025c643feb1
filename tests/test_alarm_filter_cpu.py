"""The double-precision filter in front of change detection's exact test (the walk kernel's
share_departs_filtered): it may decide only when its answer is the exact one.

The exact test (Sec. III.B, change detection; the measure is our reading): value v's share
of the window departs from its share of the Accumulator by more than pct points,
100 |MW(v) N_acc - Acc(v) N_mw| > pct N_mw N_acc.  The kernel first compares in IEEE double
precision with a margin of 2^-49 of 100 (MW N_acc + Acc N_mw) + pct N_mw N_acc, for operands
below 2^53, and leaves everything within the margin to 128-bit integers.  Python floats are
IEEE doubles with the same rounding, so the mirror below takes the same decisions; the test
drives it at, next to and far from the threshold and requires no decision to contradict the
integer test.
"""

import numpy as np


def filtered(mw, acc, n, na, pct):
    """The kernel's double branch: True / False when it decides, None when it defers."""
    if n == 0 or na == 0:
        return False
    if (mw | acc | n | na) >> 53:
        return None
    a = float(mw) * float(na)
    b = float(acc) * float(n)
    d = 100.0 * abs(a - b)
    lim = float(pct) * (float(n) * float(na))
    e = 2.0 ** -49 * (100.0 * (a + b) + lim)
    if d > lim + e:
        return True
    if d < lim - e:
        return False
    return None


def exact(mw, acc, n, na, pct):
    return n != 0 and na != 0 and 100 * abs(mw * na - acc * n) > pct * n * na


def test_filter_never_contradicts_the_exact_test():
    g = np.random.default_rng(20240)
    decided = deferred = 0
    for _ in range(40000):
        scale = int(g.integers(1, 53))
        n = int(g.integers(1, 1 << scale))
        na = n + int(g.integers(0, 1 << int(g.integers(1, 53))))
        na = min(na, (1 << 53) - 1)
        acc = int(g.integers(0, na + 1))
        pct = int(g.integers(1, 101))
        # MW(v) on or next to the threshold: 100 |mw na - acc n| = pct n na solved for mw
        target = (acc * n * 100 + pct * n * na * (1 if g.integers(0, 2) else -1)) // (100 * na)
        for mw in (target - 1, target, target + 1, int(g.integers(0, n + 1))):
            if not 0 <= mw <= n:
                continue
            f = filtered(mw, acc, n, na, pct)
            if f is None:
                deferred += 1
            else:
                decided += 1
                assert f == exact(mw, acc, n, na, pct), (mw, acc, n, na, pct)
    assert decided > 10 * deferred > 0


def test_exact_ties_are_left_to_the_integers():
    # 100 |mw na - acc n| == pct n na exactly: the double branch must not decide
    for n, na, pct in ((100, 1000, 10), (1 << 40, 1 << 45, 25), (3 << 30, 5 << 33, 50)):
        for acc in (0, na // 4, na // 2):
            num = acc * n * 100 + pct * n * na
            if num % (100 * na) == 0 and num // (100 * na) <= n:
                mw = num // (100 * na)
                assert 100 * abs(mw * na - acc * n) == pct * n * na
                assert filtered(mw, acc, n, na, pct) is None


def test_large_operands_go_to_the_integers():
    assert filtered(1 << 53, 0, 1 << 53, 1 << 54, 5) is None
    assert filtered(5, 7, 0, 10, 5) is False and filtered(5, 7, 10, 0, 5) is False
