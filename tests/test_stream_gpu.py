"""GPU parity of device-resident streams (Sec. III.B Accumulator / moving window, Sec. III.C switch).

Checked exactly against ``oracle.stream_reference`` on the same chunks: every per-chunk
histogram, the Accumulator, the moving window, and the (mode, pattern) each chunk ran with,
for several windows W, lags, sub-histogram budgets and forced modes, through both the
one-launch-per-chunk path and the persistent multi-chunk path.
"""

import numpy as np
import pytest

from oracle import oracle as O
import synthgen as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def single_stream_chunks(chunk_bytes, count=None):
    """The single stream's chunk order (Normal sigma 96/32/8/2, a degenerate and a two-spike chunk)."""
    return G.stream_chunks(chunk_bytes, count)


def mixed_chunks(seed, count, max_bytes):
    """Uneven chunk sizes (including empty and unaligned), alternating peaked and wide data."""
    g = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(g.integers(0, max_bytes))
        if k % 7 == 3:
            n = 0
        kind = k % 4
        if kind == 0:
            out.append(G.constant_bytes(n, int(g.integers(0, 256))))
        elif kind == 1:
            out.append(G.clipped_normal_bytes(n, float(g.uniform(0, 255)), float(g.uniform(1, 60)), g))
        elif kind == 2:
            out.append(G.mixture_bytes(n, float(g.uniform(0.3, 0.7)), int(g.integers(0, 256)), g))
        else:
            out.append(G.uniform_bytes(n, g))
    return out


def run_stream(hm, chunks, W, theta, S, rmax, lag, mode, many, unaligned=False):
    st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=len(chunks) + 4)
    # pack all chunks into one arena (optionally at odd offsets)
    offs, pos = [], 0
    for c in chunks:
        pos += (3 if unaligned else 0)
        offs.append(pos)
        pos += c.size
        pos = (pos + 255) // 256 * 256 if not unaligned else pos
    arena = np.zeros(pos + 16, dtype=np.uint8)
    for o, c in zip(offs, chunks):
        arena[o:o + c.size] = c
    d = dev(arena)
    base = int(d.data_ptr())
    bufs = [(base + o, c.size) for o, c in zip(offs, chunks)]
    outs = torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda")
    if many:
        st.push_many(bufs, mode=mode, d_out=outs)
    else:
        for k, (p, n) in enumerate(bufs):
            st.push(p, mode=mode, d_out=outs[k], n=n)
    snap, modes, pats = st.read(len(chunks))
    got = outs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    st.close()
    return got, snap, modes, pats


def check(hm, chunks, W=1, theta=45, S=960, rmax=8, lag=0, mode=0, many=True, unaligned=False):
    ref = O.stream_reference(chunks, W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, mode=mode)
    got, snap, modes, pats = run_stream(hm, chunks, W, theta, S, rmax, lag, mode, many, unaligned)
    tag = (W, theta, S, rmax, lag, mode, many)
    assert np.array_equal(got, ref["hists"].astype(np.int64)), tag
    assert [int(x) for x in snap.acc] == ref["acc"], tag
    assert [int(x) for x in snap.mw] == ref["mw"], tag
    assert int(snap.chunks) == len(chunks)
    assert [int(m) for m in modes] == ref["modes"], tag
    assert [list(map(int, p)) for p in pats] == ref["patterns"], tag
    # the snapshot's next decision is the decision after the last chunk
    assert int(snap.next_mode) == O.decide_mode(ref["mw"], theta)
    assert snap.next_pattern.words() == O.rule_p(ref["mw"], S, rmax)
    d = hm.diag()
    assert d.invalid_patterns == 0 and d.wait_timeouts == 0 and d.merge_timeouts == 0
    return ref


@pytest.mark.parametrize("many", [True, False])
@pytest.mark.parametrize("lag", [0, 1, 3])
def test_single_stream_order_small_chunks(hm, many, lag):
    chunks = single_stream_chunks(1 << 16)
    ref = check(hm, chunks, W=1, theta=45, S=960, rmax=8, lag=lag, many=many)
    # the switch fires right after the degenerate and the two-spike chunk
    ahist = [k for k, m in enumerate(ref["modes"]) if m == O.MODE_AHIST]
    assert ahist == [33 + lag, 50 + lag]


@pytest.mark.parametrize("W", [2, 4, 32])
def test_windows(hm, W):
    chunks = mixed_chunks(W, 40, 200_000)
    check(hm, chunks, W=W, theta=45, S=960, rmax=8, lag=0, many=True)
    check(hm, chunks, W=W, theta=30, S=2048, rmax=16, lag=2, many=True)


@pytest.mark.parametrize("S,rmax", [(960, 8), (8192, 32), (300, 64), (16384, 64), (4096, 32)])
def test_budgets(hm, S, rmax):
    chunks = mixed_chunks(S + rmax, 24, 300_000)
    check(hm, chunks, W=1, theta=45, S=S, rmax=rmax, lag=0, many=True, unaligned=True)
    check(hm, chunks, W=3, theta=20, S=S, rmax=rmax, lag=1, many=False)


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_forced_modes(hm, mode):
    chunks = mixed_chunks(50 + mode, 20, 150_000)
    check(hm, chunks, W=1, theta=45, S=960, rmax=8, lag=0, mode=mode, many=True)
    check(hm, chunks, W=2, theta=45, S=8192, rmax=32, lag=2, mode=mode, many=False)


def test_theta_edges(hm):
    # two-spike chunk: exactly 50 %: switches at theta 45 and 49, not at theta 50
    two = G.two_spike_bytes(1 << 16, G.rng(9, 1))
    chunks = [G.uniform_bytes(1 << 16, G.rng(9, 2)), two, G.uniform_bytes(1 << 16, G.rng(9, 3))]
    for theta, want in ((45, 1), (49, 1), (50, 2), (0, 1), (100, 2)):
        ref = check(hm, chunks, W=1, theta=theta, S=960, rmax=8, lag=0)
        assert ref["modes"][2] == want


def test_push_and_push_many_agree_across_calls(hm):
    # a stream continued over several calls equals one long call
    chunks = mixed_chunks(77, 30, 120_000)
    ref = O.stream_reference(chunks, W=2, theta_pct=40, S=960, rmax=8, lag=1)
    st = hm.Stream(W=2, theta_pct=40, S=960, rmax=8, lag=1, trace_cap=64)
    ds = [dev(c) if c.size else None for c in chunks]
    outs = torch.zeros((len(chunks), 256), dtype=torch.int32, device="cuda")
    bufs = [(int(x.data_ptr()) if x is not None else 0, c.size) for x, c in zip(ds, chunks)]
    st.push_many(bufs[:7], d_out=outs[:7])
    for k in range(7, 12):
        st.push(bufs[k][0], d_out=outs[k], n=bufs[k][1])
    st.push_many(bufs[12:], d_out=outs[12:])
    snap, modes, pats = st.read(len(chunks))
    assert np.array_equal(outs.cpu().numpy().astype(np.int64), ref["hists"].astype(np.int64))
    assert [int(m) for m in modes] == ref["modes"]
    assert [list(map(int, p)) for p in pats] == ref["patterns"]
    assert [int(x) for x in snap.acc] == ref["acc"]
    st.close()


def test_full_size_single_stream(hm):
    # the single stream at its real size: 66 chunks of 4 MiB, lags 0 and 1 (the scope's
    # config-2 row, with the paper's budget) and pipelined lags
    chunks = single_stream_chunks(4 << 20)
    hists = [O.hist(c) for c in chunks]
    for lag, S, rmax, theta in ((0, 960, 8, 45), (1, 960, 8, 45), (15, 8192, 32, 45), (7, 960, 8, 0)):
        ref = O.stream_reference(None, W=1, theta_pct=theta, S=S, rmax=rmax, lag=lag, hists=hists)
        got, snap, modes, pats = run_stream(hm, chunks, 1, theta, S, rmax, lag, 0, True)
        assert np.array_equal(got, ref["hists"].astype(np.int64)), lag
        assert [int(m) for m in modes] == ref["modes"], lag
        assert [list(map(int, p)) for p in pats] == ref["patterns"], lag
        assert [int(x) for x in snap.acc] == ref["acc"]


def test_long_stream_over_launch_limit(hm):
    # more chunks than one persistent launch holds: split into launches, same semantics
    chunks = [G.constant_bytes(512, k % 256) if k % 5 else G.uniform_bytes(700, G.rng(8, k)) for k in range(1100)]
    check(hm, chunks, W=1, theta=45, S=960, rmax=8, lag=2, many=True)


def test_push_many_single_chunk(hm):
    # one chunk per persistent launch, repeatedly: same semantics as one long call
    chunks = mixed_chunks(91, 9, 400_000)
    ref = O.stream_reference(chunks, W=2, theta_pct=45, S=960, rmax=8, lag=1)
    st = hm.Stream(W=2, theta_pct=45, S=960, rmax=8, lag=1, trace_cap=16)
    ds = [dev(c) if c.size else None for c in chunks]
    outs = torch.zeros((len(chunks), 256), dtype=torch.int32, device="cuda")
    for k, (x, c) in enumerate(zip(ds, chunks)):
        st.push_many([(int(x.data_ptr()) if x is not None else 0, c.size)], d_out=outs[k:k + 1])
    snap, modes, pats = st.read(len(chunks))
    assert np.array_equal(outs.cpu().numpy().astype(np.int64), ref["hists"].astype(np.int64))
    assert [int(m) for m in modes] == ref["modes"]
    assert [list(map(int, p)) for p in pats] == ref["patterns"]
    assert [int(x) for x in snap.acc] == ref["acc"]
    st.close()


@pytest.mark.parametrize("W,lag,S,rmax,theta", [(1, 0, 960, 8, 45), (1, 3, 960, 8, 45), (3, 2, 8192, 32, 45),
                                                (1, 5, 8192, 32, 0), (2, 1, 300, 64, 30)])
def test_pushes_on_alternating_hip_streams(hm, W, lag, S, rmax, theta):
    # consecutive launches of one stream on two HIP streams may overlap on the device; every
    # chunk waits for its own decision, so the results equal the sequential ones exactly
    chunks = mixed_chunks(300 + lag, 48, 200_000)
    ref = O.stream_reference(chunks, W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag)
    st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=len(chunks))
    ds = [dev(c) if c.size else None for c in chunks]
    outs = torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda")
    bufs = [(int(x.data_ptr()) if x is not None else 0, c.size) for x, c in zip(ds, chunks)]
    torch.cuda.synchronize()
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    k, call = 0, 0
    for n in (5, 1, 7, 3, 1, 9, 2, 6, 4, 10):
        if call % 3 == 1:
            for j in range(k, k + n):
                st.push(bufs[j][0], d_out=outs[j], n=bufs[j][1], stream=hs[call & 1])
        else:
            st.push_many(bufs[k:k + n], d_out=outs[k:k + n], stream=hs[call & 1])
        k += n
        call += 1
    assert k == len(chunks)
    snap, modes, pats = st.read(len(chunks), stream=hs[0])
    torch.cuda.synchronize()
    assert np.array_equal(outs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF, ref["hists"].astype(np.int64))
    assert [int(x) for x in snap.acc] == ref["acc"]
    assert [int(x) for x in snap.mw] == ref["mw"]
    assert int(snap.chunks) == len(chunks)
    assert [int(m) for m in modes] == ref["modes"]
    assert [list(map(int, p)) for p in pats] == ref["patterns"]
    d = hm.diag()
    assert d.invalid_patterns == 0 and d.wait_timeouts == 0 and d.merge_timeouts == 0
    st.close()


def test_full_size_pushes_overlapping(hm):
    # the full 66 x 4 MiB stream pushed three times over two HIP streams at the bench's lag
    chunks = single_stream_chunks(4 << 20)
    hists = [O.hist(c) for c in chunks] * 3
    lag, S, rmax, theta = 31, 8192, 32, 0
    ref = O.stream_reference(None, W=1, theta_pct=theta, S=S, rmax=rmax, lag=lag, hists=hists)
    d = dev(np.concatenate(chunks))
    base = int(d.data_ptr())
    bufs = [(base + k * (4 << 20), 4 << 20) for k in range(len(chunks))]
    outs = [torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda") for _ in range(3)]
    st = hm.Stream(W=1, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=len(hists))
    torch.cuda.synchronize()
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    for r in range(3):
        st.push_many(bufs, d_out=outs[r], stream=hs[r & 1])
    snap, modes, pats = st.read(len(hists), stream=hs[0])
    torch.cuda.synchronize()
    got = np.concatenate([o.cpu().numpy().astype(np.int64) & 0xFFFFFFFF for o in outs])
    assert np.array_equal(got, ref["hists"].astype(np.int64))
    assert [int(x) for x in snap.acc] == ref["acc"]
    assert [int(m) for m in modes] == ref["modes"]
    assert [list(map(int, p)) for p in pats] == ref["patterns"]
    dg = hm.diag()
    assert dg.invalid_patterns == 0 and dg.wait_timeouts == 0 and dg.merge_timeouts == 0
    st.close()


@pytest.mark.parametrize("frame_bytes,count", [(1 << 18, 512), (2048 * 2048, 48)])
def test_xray_frame_stream(hm, frame_bytes, count):
    # the X-ray-like frame stream (drifting mean, random width, 1 % saturated pixels): every
    # frame's histogram and the exact mode / pattern traces at the paper's theta, with the
    # pattern carried on the device, sequential (lag 0) and pipelined
    specs = G.xray_specs(count)
    frames = [G.xray_frame(t, specs[t], frame_bytes) for t in range(count)]
    hists = [O.hist(f) for f in frames]
    d = dev(np.concatenate(frames))
    base = int(d.data_ptr())
    bufs = [(base + t * frame_bytes, frame_bytes) for t in range(count)]
    # the mean's walk stays inside 57..183 and the peak bin holds 1-7 % of a frame, so the
    # paper's theta = 45 never fires on these frames; theta = 4 and 3 make the stream cross
    for lag, S, rmax, theta in ((0, 960, 8, 45), (31, 8192, 32, 4), (7, 4096, 32, 3)):
        ref = O.stream_reference(None, W=1, theta_pct=theta, S=S, rmax=rmax, lag=lag, hists=hists)
        st = hm.Stream(W=1, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=count)
        outs = torch.full((count, 256), -1, dtype=torch.int32, device="cuda")
        st.push_many(bufs, d_out=outs)
        snap, modes, pats = st.read(count)
        st.close()
        assert np.array_equal(outs.cpu().numpy().astype(np.int64), ref["hists"].astype(np.int64)), lag
        assert [int(m) for m in modes] == ref["modes"], lag
        assert [list(map(int, p)) for p in pats] == ref["patterns"], lag
        assert [int(x) for x in snap.acc] == ref["acc"], lag
        n_ahist = sum(1 for m in ref["modes"] if m == O.MODE_AHIST)
        if theta <= 4:   # narrow frames cross theta: both kernels run
            assert 0 < n_ahist < count, (theta, n_ahist)


@pytest.mark.parametrize("W,S,rmax,theta,lag", [(5, 8192, 32, 0, 3), (6, 960, 8, 30, 1), (7, 8192, 32, 45, 0),
                                                (12, 300, 64, 20, 4), (64, 2048, 16, 10, 7)])
def test_window_sizes_around_sequencer_batch(hm, W, S, rmax, theta, lag):
    # the device sequences W > 1 streams several chunks per round trip; windows shorter and
    # longer than that batch (the chunk leaving the window inside or outside the batch), many
    # small chunks that finish out of order, and only the first chunks traced (the rest are
    # published by tag alone), over two HIP streams
    chunks = mixed_chunks(900 + W, 300, 60_000)
    ref = O.stream_reference(chunks, W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag)
    traced = 40
    st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=traced)
    ds = [dev(c) if c.size else None for c in chunks]
    outs = torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda")
    bufs = [(int(x.data_ptr()) if x is not None else 0, c.size) for x, c in zip(ds, chunks)]
    torch.cuda.synchronize()
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    k, call = 0, 0
    while k < len(chunks):
        n = min(len(chunks) - k, (17, 64, 3, 100)[call % 4])
        st.push_many(bufs[k:k + n], d_out=outs[k:k + n], stream=hs[call & 1])
        k += n
        call += 1
    snap, modes, pats = st.read(traced, stream=hs[0])
    torch.cuda.synchronize()
    tag = (W, S, rmax, theta, lag)
    assert np.array_equal(outs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF, ref["hists"].astype(np.int64)), tag
    assert [int(x) for x in snap.acc] == ref["acc"], tag
    assert [int(x) for x in snap.mw] == ref["mw"], tag
    assert int(snap.chunks) == len(chunks)
    assert [int(m) for m in modes] == ref["modes"][:traced], tag
    assert [list(map(int, p)) for p in pats] == ref["patterns"][:traced], tag
    assert int(snap.next_mode) == O.decide_mode(ref["mw"], theta)
    assert snap.next_pattern.words() == O.rule_p(ref["mw"], S, rmax)
    d = hm.diag()
    assert d.invalid_patterns == 0 and d.wait_timeouts == 0 and d.merge_timeouts == 0
    st.close()


@pytest.mark.parametrize("W,lag", [(3, 1), (4, 0), (2, 6)])
def test_window_decisions_known_to_the_host(hm, W, lag):
    # with the uniform switch (theta 0, S >= 256 rmax) the host hands every chunk its
    # decision (AHist iff a chunk of the window held a byte) and nothing waits; runs of empty
    # chunks longer than the window give the per-wavefront decisions, and the traces must
    # still equal the rule's
    g = np.random.default_rng(77 + W + lag)
    chunks = []
    for k in range(90):
        n = 0 if (k // 6) % 3 == 1 else int(g.integers(1, 150_000))
        chunks.append(G.clipped_normal_bytes(n, float(g.uniform(20, 235)), float(g.uniform(2, 40)), g))
    ref = check(hm, chunks, W=W, theta=0, S=8192, rmax=32, lag=lag, many=True)
    assert len(set(ref["modes"])) == 2   # both decisions occur


@pytest.mark.parametrize("W,lag,criterion,theta,kappa", [(8, 2, 0, 0, 0), (40, 0, 0, 0, 0), (5, 9, 1, 45, 0)])
def test_window_read_between_pushes(hm, W, lag, criterion, theta, kappa):
    # with the uniform switch a window stream's launches do not walk the window (every
    # decision comes from the host); the window is summed from the ring when read.  Reads
    # after pushes of one, a few and many chunks -- runs of empty chunks among them, the
    # window only partly filled at first, pushes on two HIP streams -- must each give the
    # rule's state after that many chunks, and the decision after the last one.
    g = np.random.default_rng(900 + W + lag)
    chunks = []
    for k in range(120):
        n = 0 if (k // 7) % 4 == 2 else int(g.integers(1, 90_000))
        chunks.append(G.clipped_normal_bytes(n, float(g.uniform(10, 245)), float(g.uniform(1, 50)), g))
    S, rmax = 8192, 32
    offs = np.cumsum([0] + [(c.size + 255) // 256 * 256 for c in chunks])
    arena = np.zeros(int(offs[-1]) + 256, dtype=np.uint8)
    for o, c in zip(offs, chunks):
        arena[o:o + c.size] = c
    d = dev(arena)
    bufs = [(int(d.data_ptr()) + int(o), c.size) for o, c in zip(offs, chunks)]
    outs = torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda")
    st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=len(chunks), criterion=criterion,
                   kappa_pct=kappa)
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    n = 0
    for i, m in enumerate([1, 4, 30, 1, 1, 12, 50, 21]):
        st.push_many(bufs[n:n + m], d_out=outs[n:n + m], stream=hs[i & 1])
        n += m
        if i % 2 == 1 or n == len(chunks):
            ref = O.stream_reference(chunks[:n], W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag,
                                     criterion=criterion, kappa_pct=kappa)
            snap, modes, pats = st.read(n, stream=hs[i & 1])
            tag = (W, lag, n)
            assert int(snap.chunks) == n, tag
            assert [int(x) for x in snap.acc] == ref["acc"], tag
            assert [int(x) for x in snap.mw] == ref["mw"], tag
            assert [int(x) for x in modes] == ref["modes"], tag
            assert [list(map(int, p)) for p in pats] == ref["patterns"], tag
            # both tests fire for any non-empty window here
            want = O.MODE_AHIST if sum(ref["mw"]) > 0 else O.MODE_WAVEHIST
            assert int(snap.next_mode) == want, tag
            assert snap.next_pattern.words() == O.rule_p(ref["mw"], S, rmax), tag
    assert n == len(chunks)
    got = outs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    assert np.array_equal(got, ref["hists"].astype(np.int64))
    assert len(set(ref["modes"])) == 2
    dg = hm.diag()
    assert dg.invalid_patterns == 0 and dg.wait_timeouts == 0 and dg.merge_timeouts == 0
    st.close()


@pytest.mark.parametrize("W", [32, 256])
def test_full_size_moving_window_overlapping(hm, W):
    # the bench's moving-window streams: 66 x 4 MiB pushed three times over two HIP streams at
    # lag 31, the first push traced
    chunks = single_stream_chunks(4 << 20)
    hists = [O.hist(c) for c in chunks] * 3
    lag, S, rmax, theta = 31, 8192, 32, 0
    ref = O.stream_reference(None, W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, hists=hists)
    d = dev(np.concatenate(chunks))
    base = int(d.data_ptr())
    bufs = [(base + k * (4 << 20), 4 << 20) for k in range(len(chunks))]
    outs = [torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda") for _ in range(3)]
    st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=len(chunks))
    torch.cuda.synchronize()
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    for r in range(3):
        st.push_many(bufs, d_out=outs[r], stream=hs[r & 1])
    snap, modes, pats = st.read(len(chunks), stream=hs[0])
    torch.cuda.synchronize()
    got = np.concatenate([o.cpu().numpy().astype(np.int64) & 0xFFFFFFFF for o in outs])
    assert np.array_equal(got, ref["hists"].astype(np.int64))
    assert [int(x) for x in snap.acc] == ref["acc"]
    assert [int(x) for x in snap.mw] == ref["mw"]
    assert [int(m) for m in modes] == ref["modes"][:len(chunks)]
    assert [list(map(int, p)) for p in pats] == ref["patterns"][:len(chunks)]
    assert int(snap.next_mode) == O.decide_mode(ref["mw"], theta)
    assert snap.next_pattern.words() == O.rule_p(ref["mw"], S, rmax)
    dg = hm.diag()
    assert dg.invalid_patterns == 0 and dg.wait_timeouts == 0 and dg.merge_timeouts == 0
    st.close()


@pytest.mark.parametrize("lag,criterion,theta,kappa,S,rmax", [(0, 0, 0, 0, 8192, 32), (2, 0, 0, 0, 16384, 64),
                                                             (0, 1, 45, 0, 8192, 32), (1, 2, 30, 0, 4096, 16),
                                                             (0, 2, 0, 40, 2048, 8)])
def test_decisions_known_in_advance(hm, lag, criterion, theta, kappa, S, rmax):
    # W = 1 with a saturated budget and a test that fires for any non-empty window: the host
    # hands each chunk the decision it runs with (from the size of chunk k - 1 - lag), so no
    # chunk waits; empty chunks make some of those decisions the per-wavefront kernel.  Pushes
    # are split across launches and two HIP streams; every trace must still be the oracle's.
    chunks = mixed_chunks(1300 + lag * 7 + criterion, 140, 120_000)
    ref = O.stream_reference(chunks, W=1, theta_pct=theta, S=S, rmax=rmax, lag=lag, criterion=criterion,
                             kappa_pct=kappa)
    assert O.MODE_WAVEHIST in ref["modes"][lag + 1:] and O.MODE_AHIST in ref["modes"]
    st = hm.Stream(W=1, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=len(chunks), criterion=criterion,
                   kappa_pct=kappa)
    ds = [dev(c) if c.size else None for c in chunks]
    outs = torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda")
    bufs = [(int(x.data_ptr()) if x is not None else 0, c.size) for x, c in zip(ds, chunks)]
    torch.cuda.synchronize()
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    k, call = 0, 0
    while k < len(chunks):
        n = min(len(chunks) - k, (1, 23, 4, 50)[call % 4])
        if n == 1:
            st.push(bufs[k][0], d_out=outs[k], n=bufs[k][1], stream=hs[call & 1])
        else:
            st.push_many(bufs[k:k + n], d_out=outs[k:k + n], stream=hs[call & 1])
        k += n
        call += 1
    snap, modes, pats = st.read(len(chunks), stream=hs[0])
    torch.cuda.synchronize()
    assert np.array_equal(outs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF, ref["hists"].astype(np.int64))
    assert [int(x) for x in snap.acc] == ref["acc"]
    assert [int(x) for x in snap.mw] == ref["mw"]
    assert [int(m) for m in modes] == ref["modes"]
    assert [list(map(int, p)) for p in pats] == ref["patterns"]
    assert int(snap.next_mode) == O.decide_mode(ref["mw"], theta, criterion, kappa)
    assert snap.next_pattern.words() == O.rule_p(ref["mw"], S, rmax)
    d = hm.diag()
    assert d.invalid_patterns == 0 and d.wait_timeouts == 0 and d.merge_timeouts == 0
    st.close()


def with_empty_runs(chunks, run, at):
    """Insert `run` empty chunks before each index in `at` (windows of up to `run` chunks then
    hold no byte, so the switch picks the per-wavefront kernel)."""
    out = []
    for k, c in enumerate(chunks):
        if k in at:
            out.extend(np.zeros(0, dtype=np.uint8) for _ in range(run))
        out.append(c)
    return out


@pytest.mark.parametrize("W,lag,alarm,criterion,theta,kappa", [
    (2, 0, 0, 0, 0, 0), (3, 2, 0, 2, 30, 0), (32, 0, 5, 0, 0, 0), (5, 1, 3, 1, 100, 0), (1, 0, 4, 0, 0, 0)])
def test_window_empty_runs_and_alarms(hm, W, lag, alarm, criterion, theta, kappa):
    # A moving window (or change detection, which sequences the chunks too) with a saturated
    # budget and a test that fires for any non-empty window: runs of empty chunks longer than
    # the window empty it, so some decisions are the per-wavefront kernel.  Pushes of uneven
    # sizes over two HIP streams; every trace, the window, the Accumulator and the alarms must
    # be the oracle's.
    S, rmax = 8192, 32
    chunks = with_empty_runs(mixed_chunks(2100 + W * 3 + lag, 120, 100_000), W + 2, {30, 77})
    ref = O.stream_reference(chunks, W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, criterion=criterion,
                             kappa_pct=kappa, alarm_pct=alarm)
    assert O.MODE_WAVEHIST in ref["modes"][lag + 1:] and O.MODE_AHIST in ref["modes"]
    st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=len(chunks), criterion=criterion,
                   kappa_pct=kappa, alarm_pct=alarm)
    ds = [dev(c) if c.size else None for c in chunks]
    outs = torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda")
    bufs = [(int(x.data_ptr()) if x is not None else 0, c.size) for x, c in zip(ds, chunks)]
    torch.cuda.synchronize()
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    k, call = 0, 0
    while k < len(chunks):
        n = min(len(chunks) - k, (1, 37, 3, 66)[call % 4])
        st.push_many(bufs[k:k + n], d_out=outs[k:k + n], stream=hs[call & 1])
        k += n
        call += 1
    snap, modes, pats = st.read(len(chunks), stream=hs[0])
    alarms = st.read_alarms(len(chunks), stream=hs[0]) if alarm else None
    torch.cuda.synchronize()
    assert np.array_equal(outs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF, ref["hists"].astype(np.int64))
    assert [int(x) for x in snap.acc] == ref["acc"]
    assert [int(x) for x in snap.mw] == ref["mw"]
    assert [int(m) for m in modes] == ref["modes"]
    assert [list(map(int, p)) for p in pats] == ref["patterns"]
    assert int(snap.next_mode) == O.decide_mode(ref["mw"], theta, criterion, kappa)
    if alarm:
        assert [int(a) for a in alarms] == ref["alarms"]
        assert int(snap.alarms) == sum(ref["alarms"])
    d = hm.diag()
    assert d.invalid_patterns == 0 and d.wait_timeouts == 0 and d.merge_timeouts == 0
    st.close()


def test_window_ring_wraps(hm):
    # The sequencer's ring of recent histograms holds W + lag + 66 chunks; a chunk reuses a
    # slot only after its decision, which comes after the slot's old chunk has left the
    # window.  Push 5000 small chunks (pushes larger than one launch's 1024 chunks, over two
    # HIP streams, no synchronisation) so that the ring wraps dozens of times, and check every
    # histogram, the alarms and the final window.
    g = np.random.default_rng(515)
    # uniform bytes, every eleventh chunk empty, and bursts of a constant value (alarms)
    chunks = [np.zeros(0, dtype=np.uint8) if k % 11 == 0 else
              G.constant_bytes(int(n), 7) if k % 97 < 8 else G.uniform_bytes(int(n), g)
              for k, n in enumerate(g.integers(1, 3000, 5000))]
    W, lag, S, rmax = 7, 0, 8192, 32
    ref = O.stream_reference(chunks, W=W, theta_pct=0, S=S, rmax=rmax, lag=lag, alarm_pct=20)
    st = hm.Stream(W=W, theta_pct=0, S=S, rmax=rmax, lag=lag, trace_cap=len(chunks), alarm_pct=20)
    arena = dev(np.concatenate(chunks))
    base, pos, bufs = int(arena.data_ptr()), 0, []
    for c in chunks:
        bufs.append((base + pos, c.size))
        pos += c.size
    outs = torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    k, call = 0, 0
    while k < len(chunks):
        n = min(len(chunks) - k, (1500, 700, 2100)[call % 3])
        st.push_many(bufs[k:k + n], d_out=outs[k:k + n], stream=hs[call & 1])
        k += n
        call += 1
    snap, modes, _ = st.read(len(chunks), stream=hs[0])
    alarms = st.read_alarms(len(chunks), stream=hs[0])
    torch.cuda.synchronize()
    assert np.array_equal(outs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF, ref["hists"].astype(np.int64))
    assert [int(x) for x in snap.mw] == ref["mw"]
    assert [int(x) for x in snap.acc] == ref["acc"]
    assert [int(m) for m in modes] == ref["modes"]
    assert [int(a) for a in alarms] == ref["alarms"]
    d = hm.diag()
    assert d.invalid_patterns == 0 and d.wait_timeouts == 0 and d.merge_timeouts == 0
    st.close()


def test_known_decisions_thousands_of_tiny_chunks(hm):
    # decisions known on the host, so each workgroup takes an equal share of the launch's
    # bytes: with 3000 chunks of 0..4000 bytes (one in seven empty) a share spans hundreds of
    # chunks; pushes of uneven sizes over two HIP streams, every trace exact
    g = np.random.default_rng(31337)
    chunks = [np.zeros(0, dtype=np.uint8) if k % 7 == 3 else
              (G.constant_bytes(int(n), k % 256) if k % 5 == 0 else G.uniform_bytes(int(n), g))
              for k, n in enumerate(g.integers(1, 4000, 3000))]
    S, rmax, lag = 8192, 32, 0
    ref = O.stream_reference(chunks, W=1, theta_pct=0, S=S, rmax=rmax, lag=lag)
    st = hm.Stream(W=1, theta_pct=0, S=S, rmax=rmax, lag=lag, trace_cap=len(chunks))
    arena = dev(np.concatenate(chunks))
    base, pos, rows = int(arena.data_ptr()), 0, []
    for c in chunks:
        rows.append((base + pos, c.size))
        pos += c.size
    rows = np.array(rows, dtype=np.int64)
    outs = torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    k, call = 0, 0
    while k < len(chunks):
        n = min(len(chunks) - k, (1100, 37, 900, 1)[call % 4])
        st.push_many(rows[k:k + n], d_out=outs[k:k + n], stream=hs[call & 1])
        k += n
        call += 1
    snap, modes, pats = st.read(len(chunks), stream=hs[0])
    torch.cuda.synchronize()
    assert np.array_equal(outs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF, ref["hists"].astype(np.int64))
    assert [int(x) for x in snap.acc] == ref["acc"]
    assert [int(m) for m in modes] == ref["modes"]
    assert [list(map(int, p)) for p in pats] == ref["patterns"]
    d = hm.diag()
    assert d.invalid_patterns == 0 and d.wait_timeouts == 0 and d.merge_timeouts == 0
    st.close()

@pytest.mark.parametrize("W,lag,theta,S,rmax,alarm,pieces", [
    (32, 66, 0, 8192, 32, 0, (67, 40, 67)),            # every push within lag + 1 chunks
    (5, 9, 0, 8192, 32, 3, (10, 3, 25, 1, 10, 7)),      # a 25-chunk push falls back to the in-order plan
    (1, 12, 45, 960, 8, 0, (13, 13, 5, 40, 13)),        # data-dependent decisions, rule P rationed
    (32, 20, 45, 960, 8, 0, (21, 21, 21, 3))])
def test_decisions_from_earlier_launches(hm, W, lag, theta, S, rmax, alarm, pieces):
    # A push of at most lag + 1 chunks takes every decision from earlier launches, so its
    # chunks never wait on each other and it runs on equal byte shares while still waiting
    # for the device's decisions; longer pushes keep the in-order plan.  Two HIP streams,
    # every trace, the window, the Accumulator and the alarms exact.
    chunks = mixed_chunks(4400 + W + lag, 150, 90_000)
    ref = O.stream_reference(chunks, W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, alarm_pct=alarm)
    st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=len(chunks), alarm_pct=alarm)
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
    snap, modes, pats = st.read(len(chunks), stream=hs[0])
    alarms = st.read_alarms(len(chunks), stream=hs[0]) if alarm else None
    torch.cuda.synchronize()
    assert np.array_equal(outs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF, ref["hists"].astype(np.int64))
    assert [int(x) for x in snap.acc] == ref["acc"]
    assert [int(x) for x in snap.mw] == ref["mw"]
    assert [int(m) for m in modes] == ref["modes"]
    assert [list(map(int, p)) for p in pats] == ref["patterns"]
    if alarm:
        assert [int(a) for a in alarms] == ref["alarms"]
    d = hm.diag()
    assert d.invalid_patterns == 0 and d.wait_timeouts == 0 and d.merge_timeouts == 0
    st.close()

def test_full_size_lag0_known_decisions(hm):
    # the single stream at lag 0 (chunk k + 1's pattern from chunk k) with the tuned switch:
    # three pushes over two HIP streams, exact against the oracle
    chunks = single_stream_chunks(4 << 20)
    hists = [O.hist(c) for c in chunks] * 3
    S, rmax, theta = 8192, 32, 0
    ref = O.stream_reference(None, W=1, theta_pct=theta, S=S, rmax=rmax, lag=0, hists=hists)
    d = dev(np.concatenate(chunks))
    base = int(d.data_ptr())
    bufs = [(base + k * (4 << 20), 4 << 20) for k in range(len(chunks))]
    outs = [torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda") for _ in range(3)]
    st = hm.Stream(W=1, theta_pct=theta, S=S, rmax=rmax, lag=0, trace_cap=len(hists))
    torch.cuda.synchronize()
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    for r in range(3):
        st.push_many(bufs, d_out=outs[r], stream=hs[r & 1])
    snap, modes, pats = st.read(len(hists), stream=hs[0])
    torch.cuda.synchronize()
    got = np.concatenate([o.cpu().numpy().astype(np.int64) & 0xFFFFFFFF for o in outs])
    assert np.array_equal(got, ref["hists"].astype(np.int64))
    assert [int(x) for x in snap.acc] == ref["acc"]
    assert [int(m) for m in modes] == ref["modes"]
    assert [list(map(int, p)) for p in pats] == ref["patterns"]
    dg = hm.diag()
    assert dg.invalid_patterns == 0 and dg.wait_timeouts == 0 and dg.merge_timeouts == 0
    st.close()


def test_waiting_launches_do_not_starve(hm):
    # Chunks that wait for decisions spin on their CU.  Two launches of a stream may be in
    # flight and are dispatched together, so a launch that may wait must leave room for the
    # other: with the tuned shape forced to four workgroups per CU (more than half of what a
    # CU holds), the library still caps it.  A slow decision path (W = 32, the paper's
    # 960-entry budget, the collision criterion) over two HIP streams must finish with no
    # decision wait timing out, and every trace exact.
    chunks = single_stream_chunks(4 << 20)
    hists = [O.hist(c) for c in chunks] * 3
    W, theta, S, rmax, lag = 32, 100, 960, 8, 31
    ref = O.stream_reference(None, W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, hists=hists, criterion=1,
                             kappa_pct=3)
    d = dev(np.concatenate(chunks))
    base = int(d.data_ptr())
    bufs = [(base + k * (4 << 20), 4 << 20) for k in range(len(chunks))]
    outs = [torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda") for _ in range(3)]
    old = hm.tune_get(hm.TUNE_STREAM)
    hm.tune_set(hm.TUNE_STREAM, blocks_per_cu=4, tiles_per_wg=3)
    try:
        d0 = int(hm.diag().wait_timeouts)
        st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=len(hists), criterion=1, kappa_pct=3)
        torch.cuda.synchronize()
        hs = [torch.cuda.Stream(), torch.cuda.Stream()]
        for r in range(3):
            st.push_many(bufs, d_out=outs[r], stream=hs[r & 1])
        snap, modes, pats = st.read(len(hists), stream=hs[0])
        torch.cuda.synchronize()
        st.close()
    finally:
        hm.tune_set(hm.TUNE_STREAM, old.blocks_per_cu, old.tile_kib, old.merge_copies, old.tiles_per_wg)
    got = np.concatenate([o.cpu().numpy().astype(np.int64) & 0xFFFFFFFF for o in outs])
    assert np.array_equal(got, ref["hists"].astype(np.int64))
    assert int(hm.diag().wait_timeouts) == d0
    assert [int(m) for m in modes] == ref["modes"]
    assert [list(map(int, p)) for p in pats] == ref["patterns"]


@pytest.mark.parametrize("W,theta,lag", [(1, 45, 0), (1, 45, 1), (1, 0, 0), (4, 45, 0)])
def test_time_trace(hm, W, theta, lag):
    """The per-chunk device timeline: every traced chunk that ran has a start, a later end and
    a plausible cycle-counter rate; with decisions that depend on the data at lag 0 a chunk begins
    counting only once the chunk before it has its decision (up to the clock's sampling
    skew); untraced chunks read 0.  The traces and histograms stay exact."""
    chunks = single_stream_chunks(256 << 10, 20)
    cap = 16
    st = hm.Stream(W=W, theta_pct=theta, S=960, rmax=8, lag=lag, trace_cap=cap)
    arena = dev(np.concatenate(chunks))
    base = int(arena.data_ptr())
    bufs = [(base + k * (256 << 10), 256 << 10) for k in range(len(chunks))]
    outs = torch.zeros((len(chunks), 256), dtype=torch.int32, device="cuda")
    st.push_many(bufs[:11], d_out=outs[:11])
    st.push_many(bufs[11:], d_out=outs[11:])
    tt = st.read_times(len(chunks) + 2)
    snap, modes, pats = st.read(cap)
    st.close()
    ref = O.stream_reference(chunks, W=W, theta_pct=theta, S=960, rmax=8, lag=lag)
    assert np.array_equal(outs.cpu().numpy().astype(np.int64), ref["hists"].astype(np.int64))
    assert [int(m) for m in modes] == ref["modes"][:cap]
    assert tt.shape == (len(chunks) + 2, 3)
    assert (tt[:cap] > 0).all()
    assert (tt[cap:] == 0).all()
    assert (tt[:cap, 1] >= tt[:cap, 0]).all()
    assert ((tt[:cap, 2] >= 50) & (tt[:cap, 2] <= 10000)).all(), tt[:cap, 2]   # cycle counter, ticks/us
    if W == 1 and theta and lag == 0:
        skew = 2000   # ns
        for k in range(1, cap):
            assert int(tt[k, 0]) + skew >= int(tt[k - 1, 1]), k
