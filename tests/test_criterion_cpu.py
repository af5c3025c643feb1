"""Pins of the oracle's alternative switching criterion (the paper leaves other criteria to
future work and names one that measures the serialisation the data would cause; our reading
is the collision index sum_v p_v^2 of the moving window, the probability that two lanes of a
wavefront add into the same bin, compared with kappa percent, strict).

Expected values are closed forms worked out by hand or bounds that follow from the
mathematics (Cauchy-Schwarz, max p^2 <= sum p^2 <= max p), not the oracle's formula typed
again; planted mistakes show the pins notice plausible errors."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O


def h_of(counts):
    h = [0] * 256
    for v, c in counts.items():
        h[v] += c
    return h


@pytest.mark.parametrize("k,c", [(1, 5), (2, 3), (4, 1), (16, 7), (256, 2)])
def test_uniform_over_k_values(k, c):
    # k values, c bytes each: every p_v = 1/k, so sum p^2 = k / k^2 = 1/k
    h = h_of({v * (256 // k): c for v in range(k)})
    assert O.collision_index(h) == Fraction(1, k)


def test_two_spikes():
    assert O.collision_index(h_of({0: 7, 255: 7})) == Fraction(1, 2)
    # a and b bytes: (a^2 + b^2) / (a + b)^2
    assert O.collision_index(h_of({3: 1, 9: 3})) == Fraction(1 + 9, 16)


def test_degenerate_mixture_closed_form():
    # value v holds D bytes on top of a flat U bytes per value:
    # ((D + U)^2 + 255 U^2) / (D + 256 U)^2
    for D, U, v in [(100, 1, 0), (256, 3, 127), (0, 5, 9), (1000, 0, 200)]:
        h = [U] * 256
        h[v] += D
        expect = Fraction((D + U) ** 2 + 255 * U * U, (D + 256 * U) ** 2)
        assert O.collision_index(h) == expect


def test_empty_window():
    assert O.collision_index([0] * 256) == 0
    assert not O.collides([0] * 256, 0)


def test_bounds_from_the_mathematics():
    g = np.random.default_rng(1)
    for _ in range(200):
        h = [int(x) for x in g.integers(0, 50, 256) * (g.random(256) < g.random())]
        if sum(h) == 0:
            continue
        n = sum(h)
        pmax = Fraction(max(h), n)
        ci = O.collision_index(h)
        assert pmax * pmax <= ci <= pmax
        support = sum(1 for x in h if x)
        assert ci >= Fraction(1, support)          # Cauchy-Schwarz; equality iff flat on the support
        # relabelling the values and scaling the counts leave it unchanged
        perm = g.permutation(256)
        assert O.collision_index([h[int(i)] for i in perm]) == ci
        assert O.collision_index([3 * x for x in h]) == ci


def test_threshold_edges():
    h4 = h_of({v: 10 for v in (1, 2, 3, 4)})      # index exactly 1/4
    assert O.collides(h4, 24) and not O.collides(h4, 25)
    one = h_of({7: 9})
    assert O.collides(one, 99) and not O.collides(one, 100)


def test_decide_mode_criteria():
    # value 50 holds 856 of 1621 bytes (52.8 %), every other value 3: collision index
    # (856^2 + 255 * 9) / 1621^2 = 735031 / 2627641, about 27.97 %
    h = [3] * 256
    h[50] = 856
    n = sum(h)
    assert n == 1621 and O.collision_index(h) == Fraction(735031, 2627641)
    pmax = Fraction(max(h), n)
    ci = O.collision_index(h)
    assert Fraction(52, 100) < pmax < Fraction(53, 100) and Fraction(27, 100) < ci < Fraction(28, 100)
    A, Wv = O.MODE_AHIST, O.MODE_WAVEHIST
    assert O.decide_mode(h, 45, O.CRIT_MAXBIN, 0) == A
    assert O.decide_mode(h, 60, O.CRIT_MAXBIN, 0) == Wv
    assert O.decide_mode(h, 0, O.CRIT_COLLISION, 27) == A
    assert O.decide_mode(h, 0, O.CRIT_COLLISION, 28) == Wv
    # combined: either test suffices
    assert O.decide_mode(h, 60, O.CRIT_BOTH, 27) == A
    assert O.decide_mode(h, 45, O.CRIT_BOTH, 90) == A
    assert O.decide_mode(h, 60, O.CRIT_BOTH, 28) == Wv
    with pytest.raises(ValueError):
        O.decide_mode(h, 45, 7, 0)


def test_stream_follows_the_criterion():
    # wide chunks then a two-value chunk: with the collision criterion at 40 % the switch
    # fires after the two-value chunk (index 1/2) and not after the wide ones (index 1/256)
    wide = np.arange(256, dtype=np.uint8)
    two = np.array([5, 9] * 128, dtype=np.uint8)
    chunks = [wide, wide, two, wide]
    ref = O.stream_reference(chunks, W=1, theta_pct=100, S=960, rmax=8, lag=0, criterion=O.CRIT_COLLISION,
                             kappa_pct=40)
    assert ref["modes"] == [O.MODE_WAVEHIST, O.MODE_WAVEHIST, O.MODE_WAVEHIST, O.MODE_AHIST]
    ref = O.stream_reference(chunks, W=2, theta_pct=100, S=960, rmax=8, lag=0, criterion=O.CRIT_COLLISION,
                             kappa_pct=40)
    # W = 2 after the two-value chunk: 256 wide bytes + 256 two-value bytes,
    # index = (2 * (129^2) + 254 * 1) / 512^2, about 12.8 %: below 40
    assert ref["modes"][3] == O.MODE_WAVEHIST


def test_planted_mistakes_are_caught():
    def sum_not_squared(h):           # sum p instead of sum p^2: always 1
        n = sum(h)
        return Fraction(sum(h), n) if n else Fraction(0)

    def divides_by_n(h):              # sum h^2 / n instead of / n^2
        n = sum(h)
        return Fraction(sum(x * x for x in h), n) if n else Fraction(0)

    def max_share(h):                 # the old criterion under a new name
        n = sum(h)
        return Fraction(max(h), n) if n else Fraction(0)

    flat = h_of({v: 2 for v in range(256)})
    spikes = h_of({3: 1, 9: 3})
    assert sum_not_squared(flat) != Fraction(1, 256)
    assert divides_by_n(flat) != Fraction(1, 256)
    assert max_share(spikes) != Fraction(10, 16)
    assert O.collision_index(flat) == Fraction(1, 256) and O.collision_index(spikes) == Fraction(10, 16)
