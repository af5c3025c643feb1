"""GPU parity of change detection (Sec. III.B: the moving window compared with the Accumulator
to detect an attack or a need to reprocess; the measure is our reading, see the oracle's
``change_alarm``).

Every alarm the device raises after chunk k is checked against ``oracle.stream_reference``
on the same chunks, together with everything else the stream computes (per-chunk histograms,
Accumulator, window, the mode and pattern each chunk ran with), for windows shorter and
longer than the sequencer's batch, W = 1 (sequenced only because alarms are on), several
thresholds and lags, over two HIP streams, and at full size.
"""

import numpy as np
import pytest

from oracle import oracle as O
import synthgen as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def attack_stream(seed, count, size, start, stop, share, value):
    """Stationary clipped-Normal chunks; chunks [start, stop) carry an extra value at `share`."""
    g = np.random.default_rng(seed)
    out = []
    for k in range(count):
        c = G.clipped_normal_bytes(size, 100.0, 30.0, g)
        if start <= k < stop:
            idx = g.choice(size, int(round(share * size)), replace=False)
            c[idx] = value
        out.append(c)
    return out


def mixed(seed, count, max_bytes):
    g = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(g.integers(0, max_bytes))
        if k % 9 == 4:
            n = 0
        kind = k % 5
        if kind == 0:
            out.append(G.constant_bytes(n, int(g.integers(0, 256))))
        elif kind in (1, 2):
            out.append(G.clipped_normal_bytes(n, float(g.uniform(40, 215)), float(g.uniform(2, 50)), g))
        elif kind == 3:
            out.append(G.mixture_bytes(n, float(g.uniform(0.2, 0.8)), int(g.integers(0, 256)), g))
        else:
            out.append(G.uniform_bytes(n, g))
    return out


def run(hm, chunks, W, theta, S, rmax, lag, alarm_pct, pieces=(17, 40, 5, 64), trace=None):
    trace = len(chunks) if trace is None else trace
    st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=trace, alarm_pct=alarm_pct)
    ds = [dev(c) if c.size else None for c in chunks]
    bufs = [(int(x.data_ptr()) if x is not None else 0, c.size) for x, c in zip(ds, chunks)]
    outs = torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    k, call = 0, 0
    while k < len(chunks):
        n = min(len(chunks) - k, pieces[call % len(pieces)])
        st.push_many(bufs[k:k + n], d_out=outs[k:k + n], stream=hs[call & 1])
        k += n
        call += 1
    snap, modes, pats = st.read(trace, stream=hs[0])
    alarms = st.read_alarms(trace, stream=hs[0])
    torch.cuda.synchronize()
    got = outs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    st.close()
    return got, snap, modes, pats, alarms


def check(hm, chunks, W, alarm_pct, theta=45, S=960, rmax=8, lag=0, hists=None, trace=None, **kw):
    ref = O.stream_reference(chunks if hists is None else None, W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag,
                             hists=hists, alarm_pct=alarm_pct)
    got, snap, modes, pats, alarms = run(hm, chunks, W, theta, S, rmax, lag, alarm_pct, trace=trace, **kw)
    n = len(ref["alarms"]) if trace is None else trace
    tag = (W, alarm_pct, theta, S, rmax, lag)
    if hists is None:
        assert np.array_equal(got, ref["hists"].astype(np.int64)), tag
    assert [int(x) for x in snap.acc] == ref["acc"], tag
    assert [int(x) for x in snap.mw] == ref["mw"], tag
    assert [int(m) for m in modes] == ref["modes"][:n], tag
    assert [list(map(int, p)) for p in pats] == ref["patterns"][:n], tag
    assert [int(a) for a in alarms] == ref["alarms"][:n], tag
    hits = [k for k, a in enumerate(ref["alarms"]) if a]
    assert int(snap.alarms) == len(hits), tag
    assert int(snap.first_alarm) == (hits[0] + 1 if hits else 0), tag
    assert int(snap.last_alarm) == (hits[-1] + 1 if hits else 0), tag
    assert int(snap.next_mode) == O.decide_mode(ref["mw"], theta)
    assert snap.next_pattern.words() == O.rule_p(ref["mw"], S, rmax)
    d = hm.diag()
    assert d.invalid_patterns == 0 and d.wait_timeouts == 0 and d.merge_timeouts == 0
    return ref


@pytest.mark.parametrize("W,alarm_pct,lag,S,rmax,theta", [
    (1, 20, 0, 960, 8, 45), (2, 10, 1, 8192, 32, 0), (3, 5, 0, 960, 8, 30), (4, 30, 3, 2048, 16, 45),
    (7, 10, 2, 8192, 32, 45), (32, 5, 4, 300, 64, 20), (32, 3, 0, 960, 8, 45), (1, 15, 2, 16384, 64, 0)])
def test_alarms_match_oracle(hm, W, alarm_pct, lag, S, rmax, theta):
    chunks = mixed(700 + W * 3 + alarm_pct, 160, 80_000)
    ref = check(hm, chunks, W, alarm_pct, theta=theta, S=S, rmax=rmax, lag=lag)
    # the threshold is exercised both ways
    assert 0 < sum(ref["alarms"]) < len(chunks), (W, alarm_pct)


def test_planted_attack_is_flagged(hm):
    # stationary chunks, then ten chunks in which one value takes 30 % of the bytes, then
    # stationary again: the window departs from the Accumulator while the attack lasts
    chunks = attack_stream(5, 60, 1 << 16, 30, 40, 0.30, 250)
    ref = check(hm, chunks, 8, 10, theta=45, S=960, rmax=8, lag=0)
    # with W = 8 the value's share of the window passes 10 points above the Accumulator's
    # once four attack chunks are in it, and falls back once they leave
    assert sum(ref["alarms"][:30]) == 0
    assert sum(ref["alarms"][30:48]) >= 5
    assert sum(ref["alarms"][48:]) == 0


def test_untraced_chunks_still_counted(hm):
    # alarms past trace_cap are not traced but are counted in the snapshot
    chunks = attack_stream(9, 80, 1 << 15, 50, 70, 0.25, 3)
    ref = check(hm, chunks, 4, 8, theta=0, S=8192, rmax=32, lag=1, trace=20)
    assert sum(ref["alarms"][:20]) == 0 and sum(ref["alarms"]) > 0


def test_full_size_stream_with_alarms(hm):
    # the single stream (66 x 4 MiB) pushed three times at the bench's lag, W = 32, 4 points
    # (its window departs from its Accumulator by up to about 6 points)
    chunks = G.stream_chunks(4 << 20)
    hists = [O.hist(c) for c in chunks] * 3
    big = np.concatenate(chunks)
    d = dev(big)
    base = int(d.data_ptr())
    st = hm.Stream(W=32, theta_pct=0, S=8192, rmax=32, lag=31, trace_cap=len(hists), alarm_pct=4)
    outs = [torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda") for _ in range(3)]
    bufs = [(base + k * (4 << 20), 4 << 20) for k in range(len(chunks))]
    torch.cuda.synchronize()
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    for r in range(3):
        st.push_many(bufs, d_out=outs[r], stream=hs[r & 1])
    snap, modes, pats = st.read(len(hists), stream=hs[0])
    alarms = st.read_alarms(len(hists), stream=hs[0])
    torch.cuda.synchronize()
    ref = O.stream_reference(None, W=32, theta_pct=0, S=8192, rmax=32, lag=31, hists=hists, alarm_pct=4)
    got = np.concatenate([o.cpu().numpy().astype(np.int64) & 0xFFFFFFFF for o in outs])
    assert np.array_equal(got, ref["hists"].astype(np.int64))
    assert [int(x) for x in snap.acc] == ref["acc"]
    assert [int(x) for x in snap.mw] == ref["mw"]
    assert [int(m) for m in modes] == ref["modes"]
    assert [int(a) for a in alarms] == ref["alarms"]
    assert int(snap.alarms) == sum(ref["alarms"]) > 0
    dg = hm.diag()
    assert dg.invalid_patterns == 0 and dg.wait_timeouts == 0 and dg.merge_timeouts == 0
    st.close()


@pytest.mark.parametrize("W,alarm_pct,lag", [(5, 10, 2), (1, 15, 0), (32, 4, 7)])
def test_alarms_read_between_pushes(hm, W, alarm_pct, lag):
    # With the uniform switch each push's chunks are walked in order by a launch of its own
    # after the push, which stops at the push's last chunk; the next push's walk goes on from
    # there.  Reads after pushes of one, a few and many chunks (on two HIP streams, runs of
    # empty chunks among them) must each give the oracle's state after that many chunks:
    # alarms and their trace, the window, the Accumulator.
    chunks = attack_stream(13 + W, 120, 1 << 15, 40, 70, 0.35, 200)
    for k in range(0, len(chunks), 17):
        chunks[k] = np.zeros(0, dtype=np.uint8)
    S, rmax = 8192, 32
    ds = [dev(c) if c.size else None for c in chunks]
    bufs = [(int(x.data_ptr()) if x is not None else 0, c.size) for x, c in zip(ds, chunks)]
    outs = torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda")
    st = hm.Stream(W=W, theta_pct=0, S=S, rmax=rmax, lag=lag, trace_cap=len(chunks), alarm_pct=alarm_pct)
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    n = 0
    for i, m in enumerate([1, 7, 30, 2, 45, 35]):
        st.push_many(bufs[n:n + m], d_out=outs[n:n + m], stream=hs[i & 1])
        n += m
        if i % 2 == 1:
            ref = O.stream_reference(chunks[:n], W=W, theta_pct=0, S=S, rmax=rmax, lag=lag, alarm_pct=alarm_pct)
            snap, modes, _ = st.read(n, stream=hs[i & 1])
            alarms = st.read_alarms(n, stream=hs[i & 1])
            tag = (W, alarm_pct, lag, n)
            assert int(snap.chunks) == n, tag
            assert [int(x) for x in snap.acc] == ref["acc"], tag
            assert [int(x) for x in snap.mw] == ref["mw"], tag
            assert [int(m_) for m_ in modes] == ref["modes"], tag
            assert [int(a) for a in alarms] == ref["alarms"], tag
            hits = [k for k, a in enumerate(ref["alarms"]) if a]
            assert int(snap.alarms) == len(hits), tag
            assert int(snap.first_alarm) == (hits[0] + 1 if hits else 0), tag
            assert int(snap.last_alarm) == (hits[-1] + 1 if hits else 0), tag
    assert n == len(chunks)
    got = outs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    assert np.array_equal(got, ref["hists"].astype(np.int64))
    assert 0 < sum(ref["alarms"]) < len(chunks)
    d = hm.diag()
    assert d.invalid_patterns == 0 and d.wait_timeouts == 0 and d.merge_timeouts == 0
    st.close()


def test_read_alarms_needs_alarms_on(hm):
    st = hm.Stream(W=4, theta_pct=45, S=960, rmax=8, lag=0, trace_cap=8)
    with pytest.raises(hm.HistError):
        st.read_alarms(8)
    st.close()
