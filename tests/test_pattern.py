"""Pins for the oracle's pattern rules, degeneracy decision and stream semantics.

* PAPER960: only the facts the paper states (Sec. III.A and the discussion of
  Table 2) pin it: length 960, eight sub-bins for value 127 (the most), one
  sub-bin for the first bin.
* Rule P (pattern from past histograms; the paper gives no rule, Sec. III.B):
  closed forms for one-hot, flat and two-spike histograms plus structural
  invariants.  Beyond those, parity with the paper is unpinned.
* Degeneracy (Sec. III.C): closed forms (all-equal, uniform, the exact 50 %
  two-spike edge, Normal max-bin share from the error function).
* Streams (Sec. III.B): Accumulator = running sum, MW_k = Acc_k - Acc_{k-W},
  and the mode sequence of hand-built streams.
"""

import json
import math
import os
import random

import numpy as np
import pytest

from oracle import oracle as O
import synthgen as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def facts():
    with open(os.path.join(GOLDEN, "paper_facts.json")) as f:
        return json.load(f)


def rs(words):
    return [O.pat_r(w) for w in words]


def bases(words):
    return [O.pat_base(w) for w in words]


# ---------------------------------------------------------------- PAPER960

def test_paper960_matches_stated_facts():
    f = facts()
    w = O.pattern_paper960()
    r = rs(w)
    assert sum(r) == f["paper_pattern_length"] == O.pattern_total(w)
    assert max(r) == f["paper_pattern_max_subbins"]
    assert r[f["paper_pattern_max_value"]] == f["paper_pattern_max_subbins"]
    assert r[0] == f["paper_pattern_first_bin_subbins"]
    assert r[f["first_bin_value_example"]] == 1
    assert O.pattern_valid(w, 960, 8)


def test_identity_and_flat_closed_forms():
    w = O.pattern_identity()
    assert rs(w) == [1] * 256 and bases(w) == list(range(256))
    assert O.pattern_valid(w, 256, 1)
    w = O.pattern_flat(32)
    assert rs(w) == [32] * 256 and bases(w) == [32 * b for b in range(256)]
    assert O.pattern_valid(w, 8192, 32) and not O.pattern_valid(w, 8191, 32)


# ---------------------------------------------------------------- validity

def test_validity_rejects():
    good = O.pattern_identity()
    assert O.pattern_valid(good, 256, 1)
    bad = list(good)
    bad[3] = O.pat_word(2, 1)                     # overlaps value 2
    assert not O.pattern_valid(bad, 256, 1)
    bad = list(good)
    bad[255] = O.pat_word(255, 2)                 # runs past S
    assert not O.pattern_valid(bad, 256, 2)
    assert O.pattern_valid(bad, 257, 2)
    assert not O.pattern_valid(O.pattern_flat(4), 1024, 2)   # r above rmax
    bad = list(good)
    bad[7] = good[7] | (1 << 24)                  # stray high bits
    assert not O.pattern_valid(bad, 256, 1)
    with pytest.raises(ValueError):
        O.pat_word(0, 3)                          # r not a power of two
    assert not O.pattern_valid(good[:255], 256, 1)


# ---------------------------------------------------------------- rule P closed forms

@pytest.mark.parametrize("v", [0, 1, 127, 200, 255])
@pytest.mark.parametrize("S,rmax", [(960, 8), (4096, 32), (2048, 64), (300, 16)])
def test_rule_p_one_hot(v, S, rmax):
    h = [0] * 256
    h[v] = 12345
    w = O.rule_p(h, S, rmax)
    r = rs(w)
    assert r[v] == rmax and sum(r) == 255 + rmax
    assert all(r[b] == 1 for b in range(256) if b != v)
    assert O.pat_base(w[v]) == 0                  # r descending puts the spike first
    assert O.pattern_valid(w, S, rmax)


def test_rule_p_flat_gives_two():
    # flat histogram at S = 960, rmax = 8: t = 9 gives r = 2 (sum 512), t = 10 gives 4 (sum 1024 > 960)
    w = O.rule_p([1000] * 256, 960, 8)
    assert rs(w) == [2] * 256
    assert bases(w) == [2 * b for b in range(256)]


@pytest.mark.parametrize("S,rmax", [(8192, 32), (16384, 64), (4096, 16), (256, 1), (9000, 32)])
def test_rule_p_saturated_budget(S, rmax):
    # 256 * rmax <= S: every value gets rmax whatever the histogram, laid out in value order
    for h in ([7] * 256, [0] * 256, [0] * 255 + [99]):
        w = O.rule_p(h, S, rmax)
        assert rs(w) == [rmax] * 256
        assert bases(w) == [rmax * b for b in range(256)]


def test_rule_p_just_below_saturation():
    # S = 256 * 32 - 1: the empty values keep one sub-bin, the rest reach rmax
    h = [5] * 200 + [0] * 56
    w = O.rule_p(h, 8191, 32)
    r = rs(w)
    assert r[:200] == [32] * 200 and r[200:] == [1] * 56


def test_rule_p_two_spike():
    h = [0] * 256
    h[0] = h[255] = 1 << 21
    w = O.rule_p(h, 960, 8)
    r = rs(w)
    assert r[0] == r[255] == 8 and sum(r) == 254 + 16
    assert bases(w)[0] == 0 and bases(w)[255] == 8


def test_rule_p_empty_histogram():
    w = O.rule_p([0] * 256, 960, 8)
    assert rs(w) == [1] * 256 and bases(w) == list(range(256))


def test_rule_p_budget_256_forces_identity():
    g = np.random.default_rng(3)
    w = O.rule_p(g.integers(0, 1000, 256).tolist(), 256, 64)
    assert rs(w) == [1] * 256


def test_rule_p_hand_example():
    # h = 3/4 of the mass at value 9, 1/4 at value 4, S = 264, rmax = 8.
    # t = 2: r9 = ceil(3) -> 4, r4 = ceil(1) -> 1: sum 259 (ok)
    # t = 3: r9 = ceil(6) -> 8, r4 = ceil(2) -> 2: sum 264 (ok)
    # t = 4: r9 = 8 (cap), r4 = 4: sum 266 > 264 -> stop at t = 3
    h = [0] * 256
    h[9], h[4] = 300, 100
    w = O.rule_p(h, 264, 8)
    r = rs(w)
    assert r[9] == 8 and r[4] == 2 and sum(r) == 264
    # layout: value 9 (r 8) at 0, value 4 (r 2) at 8, then the r = 1 values in value order
    assert O.pat_base(w[9]) == 0 and O.pat_base(w[4]) == 8
    assert O.pat_base(w[0]) == 10 and O.pat_base(w[5]) == 14 and O.pat_base(w[255]) == 263


@pytest.mark.parametrize("seed", range(40))
def test_rule_p_invariants(seed):
    rnd = random.Random(seed)
    kind = seed % 4
    if kind == 0:
        h = [rnd.randrange(0, 10 ** rnd.randrange(1, 7)) for _ in range(256)]
    elif kind == 1:
        h = [0] * 256
        for _ in range(rnd.randrange(1, 6)):
            h[rnd.randrange(256)] += rnd.randrange(1, 1 << 30)
    elif kind == 2:
        x = G.clipped_normal_bytes(1 << 16, rnd.uniform(0, 255), rnd.uniform(1, 60), G.rng(97, seed))
        h = list(map(int, O.hist(x)))
    else:
        h = [rnd.randrange(0, 1 << 40) for _ in range(256)]
    S = rnd.choice([256, 300, 960, 2048, 8192, 16384])
    rmax = rnd.choice([1, 2, 4, 8, 16, 32, 64])
    w = O.rule_p(h, S, rmax)
    r, b = rs(w), bases(w)
    assert O.pattern_valid(w, S, rmax)
    assert sum(r) <= S
    assert all(x & (x - 1) == 0 and 1 <= x <= rmax for x in r)
    assert all(b[v] % r[v] == 0 for v in range(256))           # buddy alignment
    for i in range(256):                                       # monotone in h
        for j in range(256):
            if h[i] >= h[j]:
                assert r[i] >= r[j]
    # ranges tile [0, sum r) exactly, in (r desc, value asc) order
    order = sorted(range(256), key=lambda v: (-r[v], v))
    pos = 0
    for v in order:
        assert b[v] == pos
        pos += r[v]


def test_rule_p_scale_invariance():
    # only the shares h / N matter
    rnd = random.Random(11)
    h = [rnd.randrange(0, 5000) for _ in range(256)]
    assert O.rule_p(h, 960, 8) == O.rule_p([7 * x for x in h], 960, 8)


# ---------------------------------------------------------------- degeneracy

def test_degeneracy_closed_forms():
    all_v = [0] * 256
    all_v[127] = 4 << 20
    assert O.decide_mode(all_v, 45) == O.MODE_AHIST
    flat = [4096] * 256
    assert O.decide_mode(flat, 45) == O.MODE_WAVEHIST
    assert O.decide_mode(flat, 0) == O.MODE_AHIST            # theta 0: any mass exceeds it
    two = [0] * 256
    two[0] = two[255] = 1 << 21
    assert O.decide_mode(two, 45) == O.MODE_AHIST            # 50 % > 45 %
    assert O.decide_mode(two, 50) == O.MODE_WAVEHIST         # "exceed" is strict
    assert O.decide_mode([0] * 256, 45) == O.MODE_WAVEHIST   # empty window


def test_theta_default_in_paper_range():
    lo, hi = facts()["theta_range_pct"]
    assert lo <= 45 <= hi


@pytest.mark.parametrize("sigma", [2.0, 8.0, 32.0, 96.0])
def test_normal_bin_shares(sigma):
    # clip(rint(128 + sigma z), 0, 255): the central bin holds P(|z| < 0.5 / sigma); the clipped
    # edge bins hold the tails P(128 + sigma z >= 254.5) and P(128 + sigma z < 0.5)
    s2 = sigma * math.sqrt(2.0)
    p_mid = math.erf(0.5 / s2)
    p_hi = 0.5 * math.erfc((254.5 - 128.0) / s2)
    p_lo = 0.5 * math.erfc((128.0 - 0.5) / s2)
    n = 1 << 22
    h = O.hist(G.clipped_normal_bytes(n, 128.0, sigma, G.rng(96, int(sigma))))
    for b, p in ((128, p_mid), (255, p_hi), (0, p_lo)):
        assert abs(int(h[b]) / n - p) <= 5.0 * math.sqrt(p * (1 - p) / n) + 2e-6, (b, p)
    # the largest share stays far below the 40-50 % critical degeneracy
    assert int(h.max()) / n < 0.25
    assert O.decide_mode(list(map(int, h)), 45) == O.MODE_WAVEHIST


# ---------------------------------------------------------------- streams

def _h_at(v, n):
    h = [0] * 256
    h[v] = n
    return h


def test_stream_modes_lag0_and_lag1():
    uni = [16] * 256
    deg = _h_at(127, 4096)
    hs = [uni, deg, uni, uni]
    r0 = O.stream_reference(None, W=1, theta_pct=45, S=960, rmax=8, lag=0, hists=hs)
    W_, A_ = O.MODE_WAVEHIST, O.MODE_AHIST
    assert r0["modes"] == [W_, W_, A_, W_]
    assert r0["patterns"][0] == O.pattern_identity()
    assert r0["patterns"][2] == O.rule_p(deg, 960, 8)
    assert rs(r0["patterns"][2])[127] == 8
    r1 = O.stream_reference(None, W=1, theta_pct=45, S=960, rmax=8, lag=1, hists=hs)
    assert r1["modes"] == [W_, W_, W_, A_]
    assert r1["patterns"][1] == O.pattern_identity()
    assert r1["patterns"][3] == O.rule_p(deg, 960, 8)
    forced = O.stream_reference(None, lag=0, mode=O.MODE_AHIST, hists=hs)
    assert forced["modes"] == [A_] * 4
    assert forced["patterns"] == r0["patterns"]


def test_stream_window_two_dilutes_degeneracy():
    uni = [16] * 256                    # 4096 bytes
    deg = _h_at(127, 4096)
    hs = [uni, deg, uni, uni]
    # W = 2: after the degenerate chunk, MW = uni + deg -> share (16 + 4096) / 8192 = 50.2 % > 45 %
    r = O.stream_reference(None, W=2, theta_pct=45, lag=0, hists=hs)
    assert r["modes"] == [2, 2, 1, 1]
    # theta 60: W = 1 sees 100 % after the degenerate chunk, W = 2 only 50.2 %
    r = O.stream_reference(None, W=1, theta_pct=60, lag=0, hists=hs)
    assert r["modes"] == [2, 2, 1, 2]
    r = O.stream_reference(None, W=2, theta_pct=60, lag=0, hists=hs)
    assert r["modes"] == [2, 2, 2, 2]


@pytest.mark.parametrize("W", [1, 2, 3, 7])
def test_stream_accumulator_and_window(W):
    rnd = random.Random(W)
    hs = [[rnd.randrange(0, 100) for _ in range(256)] for _ in range(11)]
    r = O.stream_reference(None, W=W, hists=hs)
    acc = [0] * 256
    accs = []
    for h in hs:
        acc = [a + b for a, b in zip(acc, h)]
        accs.append(acc)
    assert r["acc"] == accs[-1]
    k = len(hs) - 1
    lo = accs[k - W] if k - W >= 0 else [0] * 256
    assert r["mw"] == [a - b for a, b in zip(accs[k], lo)]


def test_stream_chunks_recount():
    chunks = [G.constant_bytes(100, 3), G.ramp_bytes(512)]
    r = O.stream_reference(chunks)
    assert int(r["hists"][0][3]) == 100 and int(r["hists"][1].sum()) == 512
    assert r["acc"][3] == 100 + 2


def test_single_stream_trace_shape():
    # the single stream: switch right after the degenerate chunk and the two-spike chunk
    specs = G.stream_specs()
    n = 4096
    hs = []
    for k, s in enumerate(specs):
        if s.kind == "degenerate":
            hs.append(_h_at(127, n))
        elif s.kind == "twospike":
            h = [0] * 256
            h[0] = h[255] = n // 2
            hs.append(h)
        else:
            hs.append([n // 256] * 256)      # stand-in for a wide Normal chunk
    r = O.stream_reference(None, W=1, theta_pct=45, lag=0, hists=hs)
    ahist_at = [k for k, m in enumerate(r["modes"]) if m == O.MODE_AHIST]
    deg_k = [k for k, s in enumerate(specs) if s.kind in ("degenerate", "twospike")]
    assert ahist_at == [k + 1 for k in deg_k]


# ---------------------------------------------------------------- rule P rounding (hand-worked)

def _rounding_cases():
    with open(os.path.join(GOLDEN, "rule_p_rounding.json")) as f:
        return json.load(f)["cases"]


def _check_rounding_case(case):
    h = [0] * 256
    for v, n in case["spikes"].items():
        h[int(v)] = n
    w = O.rule_p(h, case["S"], case["rmax"])
    r = rs(w)
    want = [case["r_other"]] * 256
    for v, x in case["r"].items():
        want[int(v)] = x
    assert r == want
    assert sum(r) == case["sum_r"]
    for v, b in case["base"].items():
        assert O.pat_base(w[int(v)]) == b


@pytest.mark.parametrize("i", range(2))
def test_rule_p_rounding_hand_cases(i):
    # the scale t wins with shares such as 2.5 and 3.3: ceil, floor and round give
    # different sub-bin counts, so these pin the ceiling of step 2 of rule P
    _check_rounding_case(_rounding_cases()[i])


@pytest.mark.parametrize("planted", ["floor", "round_half_up", "no_pow2ceil"])
def test_rule_p_planted_rounding_is_caught(monkeypatch, planted):
    # plant a plausible mistake in the oracle's rounding and check that a pin fails
    if planted == "floor":
        monkeypatch.setattr(O, "_ceil_div", lambda a, b: a // b)
    elif planted == "round_half_up":
        monkeypatch.setattr(O, "_ceil_div", lambda a, b: (2 * a + b) // (2 * b))
    else:
        monkeypatch.setattr(O, "_pow2ceil", lambda x: x)
    failed = 0
    for case in _rounding_cases():
        try:
            _check_rounding_case(case)
        except (AssertionError, ValueError):   # a wrong count, or an invalid pattern
            failed += 1
    assert failed >= 1
