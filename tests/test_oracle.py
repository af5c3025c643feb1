"""Pins for the histogram oracle: brute force, closed forms, invariants, library special cases.

The oracle is the plain definition out[b] = #{i : in[i] == b} (Sec. III.A,
exactness per Sec. I).  Nothing here compares the oracle with itself: each
check is fixed by mathematics or by an independent library routine.
"""

import collections
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
import synthgen as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def facts():
    with open(os.path.join(GOLDEN, "paper_facts.json")) as f:
        return json.load(f)


def test_every_one_byte_input():
    # all 256 one-byte inputs: a unit vector at the byte's value
    arena = np.arange(256, dtype=np.uint8)
    out = O.hist_many(arena, np.arange(256), np.ones(256))
    assert np.array_equal(out, np.eye(256, dtype=np.uint64))
    for v in (0, 1, 127, 255):
        assert O.hist_py([v]) == [1 if b == v else 0 for b in range(256)]


def test_every_two_byte_input():
    # all 65,536 two-byte inputs (a, b): out has +1 at a and +1 at b
    a = np.repeat(np.arange(256, dtype=np.uint8), 256)
    b = np.tile(np.arange(256, dtype=np.uint8), 256)
    arena = np.stack([a, b], axis=1).reshape(-1)
    out = O.hist_many(arena, np.arange(65536) * 2, np.full(65536, 2))
    expect = np.zeros((65536, 256), dtype=np.uint64)
    rows = np.arange(65536)
    np.add.at(expect, (rows, a.astype(np.int64)), 1)
    np.add.at(expect, (rows, b.astype(np.int64)), 1)
    assert np.array_equal(out, expect)


@pytest.mark.parametrize("seed", range(20))
def test_tiny_random_against_counter(seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(0, 65))
    x = g.integers(0, 256, size=n, dtype=np.uint8)
    c = collections.Counter(int(v) for v in x)          # independent library routine
    expect = [c.get(b, 0) for b in range(256)]
    assert list(map(int, O.hist(x))) == expect
    assert O.hist_py(x) == expect


@pytest.mark.parametrize("n", [0, 1, 255, 256, 257, 1000, 65537])
@pytest.mark.parametrize("v", [0, 1, 127, 255])
def test_all_equal_closed_form(n, v):
    out = O.hist(G.constant_bytes(n, v))
    expect = np.zeros(256, dtype=np.uint64)
    expect[v] = n
    assert np.array_equal(out, expect)


@pytest.mark.parametrize("n", [0, 1, 255, 256, 257, 4096 + 77, 1 << 20])
def test_ramp_closed_form(n):
    out = O.hist(G.ramp_bytes(n))
    q, r = divmod(n, 256)
    expect = np.array([q + (1 if b < r else 0) for b in range(256)], dtype=np.uint64)
    assert np.array_equal(out, expect)


@pytest.mark.parametrize("n", [2, 4096, 4 << 20])
def test_two_spike_closed_form(n):
    out = O.hist(G.two_spike_bytes(n, G.rng(99, n)))
    assert int(out[0]) == n // 2 and int(out[255]) == n - n // 2
    assert int(out[1:255].sum()) == 0


def test_bincount_and_sum_invariant():
    x = G.image_1mib()
    out = O.hist(x)
    assert np.array_equal(out, np.bincount(x, minlength=256).astype(np.uint64))
    assert int(out.sum()) == x.size


def test_additivity():
    # O(a || b) = O(a) + O(b): pins accumulation, tile splits and batch splits
    g = np.random.default_rng(5)
    a = g.integers(0, 256, size=12345, dtype=np.uint8)
    b = G.clipped_normal_bytes(54321, 100.0, 7.0, G.rng(98, 1))
    assert np.array_equal(O.hist(np.concatenate([a, b])), O.hist(a) + O.hist(b))


def test_threaded_timing_path_matches():
    x = G.clipped_normal_bytes(3 << 20, 128.0, 20.0, G.rng(98, 2))
    ref = np.bincount(x, minlength=256).astype(np.uint64)
    for t in (1, 2, 3, 8):
        secs, out = O.hist_timed(x, t)
        assert secs >= 0.0
        assert np.array_equal(out, ref)


def test_hist_many_rejects_out_of_arena():
    with pytest.raises(ValueError):
        O.hist_many(np.zeros(10, np.uint8), [5], [6])


def test_pixel_range_fact():
    f = facts()
    assert (f["pixel_min"], f["pixel_max"], f["bins"]) == (0, 255, 256)
    # every byte value lands in its own bin
    assert np.array_equal(O.hist(np.arange(256, dtype=np.uint8)), np.ones(256, np.uint64))


def test_planted_mistakes_are_caught():
    # a plausible mistake in a counting loop (off-by-one bin, dropped last byte)
    # must fail the closed forms above; check that the closed forms notice them.
    def off_by_one(x):
        out = [0] * 256
        for v in x:
            out[(int(v) + 1) % 256] += 1
        return out

    def drop_last(x):
        return O.hist_py(list(x)[:-1])

    x = G.ramp_bytes(300)
    q, r = divmod(300, 256)
    expect = [q + (1 if b < r else 0) for b in range(256)]
    assert off_by_one(x) != expect
    assert drop_last(x) != expect
    assert O.hist_py(x) == expect
