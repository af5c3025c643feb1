"""Seeded generators: determinism, recorded digests, and distribution sanity."""

import json
import math
import os

import numpy as np
import pytest

import synthgen as G
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_determinism():
    a = G.stream_chunk(3, G.ChunkSpec("normal", 8.0), 1 << 16)
    b = G.stream_chunk(3, G.ChunkSpec("normal", 8.0), 1 << 16)
    c = G.stream_chunk(4, G.ChunkSpec("normal", 8.0), 1 << 16)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_recorded_digests():
    with open(os.path.join(GOLDEN, "gen_digests.json")) as f:
        rec = json.load(f)
    got = {
        "image_1mib": G.digest(G.image_1mib()),
        "stream_chunk0_64k": G.digest(G.stream_chunk(0, G.stream_specs()[0], 1 << 16)),
        "xray_frame0_64k": G.digest(G.xray_frame(0, G.xray_specs(1)[0], 1 << 16)),
        "batch_specs_16": G.digest(np.array([(s.w, s.h) for s in G.batch_specs(16)], dtype=np.int64)),
    }
    assert got == rec["digests"]


def test_uniform_and_ramp():
    x = G.image_1mib()
    assert x.size == 1 << 20 and x.dtype == np.uint8
    assert abs(float(x.mean()) - 127.5) < 0.5
    h = O.hist(x)
    assert int(h.min()) > 3700 and int(h.max()) < 4500
    r = G.ramp_bytes(1000)
    assert r[0] == 0 and r[255] == 255 and r[256] == 0 and r[999] == 999 % 256


def test_two_spike_and_mixture_exact():
    x = G.two_spike_bytes(4 << 20, G.rng(2, 49))
    h = O.hist(x)
    assert int(h[0]) == 2 << 20 and int(h[255]) == 2 << 20
    n = 1 << 20
    m = G.mixture_bytes(n, 0.9, 200, G.rng(4, 7))
    k = int(round(0.9 * n))
    h = O.hist(m)
    # k forced positions plus about 1/256 of the rest drawn uniformly
    assert k <= int(h[200]) <= k + 3 * (n - k) // 256 + 100


def test_stream_specs_order():
    s = G.stream_specs()
    assert len(s) == 66
    assert [x.sigma for x in s[:16]] == [96.0] * 16
    assert s[32].kind == "degenerate" and s[49].kind == "twospike"
    assert [x.sigma for x in s[50:]] == [2.0] * 16


def test_xray_frames():
    specs = G.xray_specs(512)
    assert len(specs) == 512
    mus = np.array([s.mu for s in specs])
    sig = np.array([s.sigma for s in specs])
    assert mus.min() >= 0 and mus.max() <= 255 and sig.min() >= 6 and sig.max() <= 40
    steps = np.diff(mus)
    inner = (mus[:-1] > 20) & (mus[:-1] < 235)
    assert abs(float(steps[inner].std()) - 4.0) < 0.6
    f = G.xray_frame(0, specs[0], 1 << 18)
    k = int(round(0.01 * f.size))
    assert int(O.hist(f)[255]) >= k


def test_batch_specs():
    specs = G.batch_specs(4096)
    w = np.array([s.w for s in specs])
    h = np.array([s.h for s in specs])
    assert w.min() >= 64 and w.max() <= 4096 and h.min() >= 64 and h.max() <= 4096
    mean = float((w * h).mean())
    # E[w h] = E[w]^2 with E[w] = (4096 - 64) / ln 64
    ew = (4096 - 64) / math.log(64)
    assert abs(mean / (ew * ew) - 1.0) < 0.1
    kinds = {s.kind for s in specs}
    assert kinds == {"uniform", "normal", "spike"}


def test_batch_arena_alignment():
    specs = G.batch_specs(8)
    arena, off, sz = G.batch_arena(specs, align=256)
    assert all(int(o) % 256 == 0 for o in off)
    assert int(off[-1] + sz[-1]) == arena.size
    packed, off1, _ = G.batch_arena(specs, align=1)
    assert int(off1[1]) == specs[0].size
    for j in range(8):
        assert np.array_equal(arena[int(off[j]):int(off[j] + sz[j])], packed[int(off1[j]):int(off1[j] + sz[j])])


def test_serve_requests():
    reqs = G.serve_requests(1000.0, 2.0, pool_bytes=64 << 20)
    assert 1800 < len(reqs) < 2200
    sizes = np.array([r.size for r in reqs])
    assert sizes.min() >= 4096 and sizes.max() <= 64 << 20
    assert all(0 <= r.stream_id < 64 for r in reqs)
    assert all(r.offset + r.size <= 64 << 20 for r in reqs)
    med = float(np.median(sizes))
    assert 256 << 10 < med < 1 << 20           # log-uniform median: sqrt(4 KiB * 64 MiB) = 512 KiB
