"""GPU parity of the alternative switching criterion (the collision index of the moving window,
our reading of the criterion the paper leaves to future work; see the oracle's
``collision_index``) and of the combined test (either criterion).

The kernel each chunk ran with, the pattern, every per-chunk histogram, the Accumulator and
the window are checked exactly against ``oracle.stream_reference`` with the same criterion:
W = 1 (decided in each chunk's own epilogue) and W > 1 (decided by the device's sequencer),
with and without change detection, over two HIP streams, and at full size.
"""

import numpy as np
import pytest

from oracle import oracle as O
import synthgen as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


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


def run_and_check(hm, chunks, W, theta, S, rmax, lag, criterion, kappa, alarm_pct=0, hists=None,
                  pieces=(17, 40, 5, 64)):
    ref = O.stream_reference(chunks if hists is None else None, W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag,
                             hists=hists, criterion=criterion, kappa_pct=kappa, alarm_pct=alarm_pct)
    n = len(ref["modes"])
    st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=n, alarm_pct=alarm_pct,
                   criterion=criterion, kappa_pct=kappa)
    if hists is None:
        ds = [dev(c) if c.size else None for c in chunks]
        bufs = [(int(x.data_ptr()) if x is not None else 0, c.size) for x, c in zip(ds, chunks)]
    else:
        ds = [dev(np.concatenate(chunks))]
        base, size = int(ds[0].data_ptr()), chunks[0].size
        bufs = [(base + (k % len(chunks)) * size, size) for k in range(n)]
    outs = torch.full((n, 256), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    hs = [torch.cuda.Stream(), torch.cuda.Stream()]
    k, call = 0, 0
    while k < n:
        m = min(n - k, pieces[call % len(pieces)])
        st.push_many(bufs[k:k + m], d_out=outs[k:k + m], stream=hs[call & 1])
        k += m
        call += 1
    snap, modes, pats = st.read(n, stream=hs[0])
    alarms = st.read_alarms(n, stream=hs[0]) if alarm_pct else None
    torch.cuda.synchronize()
    tag = (W, criterion, kappa, theta, lag, alarm_pct)
    assert np.array_equal(outs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF, ref["hists"].astype(np.int64)), tag
    assert [int(x) for x in snap.acc] == ref["acc"], tag
    assert [int(x) for x in snap.mw] == ref["mw"], tag
    assert [int(m) for m in modes] == ref["modes"], tag
    assert [list(map(int, p)) for p in pats] == ref["patterns"], tag
    assert int(snap.next_mode) == O.decide_mode(ref["mw"], theta, criterion, kappa), tag
    if alarm_pct:
        assert [int(a) for a in alarms] == ref["alarms"], tag
    d = hm.diag()
    assert d.invalid_patterns == 0 and d.wait_timeouts == 0 and d.merge_timeouts == 0
    st.close()
    return ref


@pytest.mark.parametrize("W,criterion,kappa,theta,lag", [
    (1, O.CRIT_COLLISION, 5, 100, 0), (1, O.CRIT_BOTH, 20, 45, 2), (3, O.CRIT_COLLISION, 10, 100, 1),
    (5, O.CRIT_BOTH, 3, 60, 0), (32, O.CRIT_COLLISION, 2, 100, 3), (32, O.CRIT_BOTH, 4, 45, 0)])
def test_criterion_matches_oracle(hm, W, criterion, kappa, theta, lag):
    chunks = mixed(1000 + W * 7 + kappa, 160, 80_000)
    ref = run_and_check(hm, chunks, W, theta, 960, 8, lag, criterion, kappa)
    # the criterion decides both ways, and differs from the paper's test somewhere
    ahist = sum(1 for m in ref["modes"] if m == O.MODE_AHIST)
    assert 0 < ahist < len(chunks)
    plain = O.stream_reference(chunks, W=W, theta_pct=theta, S=960, rmax=8, lag=lag)
    assert plain["modes"] != ref["modes"]


def test_criterion_with_change_detection(hm):
    chunks = mixed(77, 160, 80_000)
    run_and_check(hm, chunks, 7, 100, 8192, 32, 1, O.CRIT_COLLISION, 6, alarm_pct=10)


@pytest.mark.parametrize("W,kappa", [(1, 10), (32, 3)])
def test_full_size_stream_collision(hm, W, kappa):
    # the single stream (66 x 4 MiB) pushed three times at the bench's lag
    chunks = G.stream_chunks(4 << 20)
    hists = [O.hist(c) for c in chunks] * 3
    ref = run_and_check(hm, chunks, W, 100, 8192, 32, 31, O.CRIT_COLLISION, kappa, hists=hists,
                        pieces=(66,))
    ahist = sum(1 for m in ref["modes"] if m == O.MODE_AHIST)
    assert 0 < ahist < len(hists)
