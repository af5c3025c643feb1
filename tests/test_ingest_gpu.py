"""GPU parity of host-ingest streams (Sec. III.B pipelined stream): chunks copied from host
memory and pushed over 1..8 HIP streams give exactly the oracle's per-chunk histograms,
Accumulator, moving window and mode / pattern traces, as does the sequential variant (a
sync after every push)."""

import numpy as np
import pytest

from oracle import oracle as O
import synthgen as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def chunks_mixed(seed, count, max_bytes):
    g = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(g.integers(0, max_bytes))
        if k % 9 == 4:
            n = 0
        if k % 3 == 0:
            out.append(G.constant_bytes(n, int(g.integers(0, 256))))
        elif k % 3 == 1:
            out.append(G.clipped_normal_bytes(n, float(g.uniform(0, 255)), float(g.uniform(1, 40)), g))
        else:
            out.append(G.uniform_bytes(n, g))
    return out


def pinned(a: np.ndarray):
    t = torch.empty(a.size, dtype=torch.uint8, pin_memory=True)
    t.numpy()[:] = a
    return t


def run(hm, chunks, n_hip, W, theta, S, rmax, lag, sequential=False, source="pinned", extra=None):
    slot = max(1, max(c.size for c in chunks))
    ing = hm.Ingest(n_hip_streams=n_hip, slot_bytes=slot)
    st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=len(chunks), **(extra or {}))
    outs = torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    hosts = [pinned(c) if source == "pinned" else c for c in chunks]
    for k, h in enumerate(hosts):
        ing.push(st, h, d_out=outs[k], n=chunks[k].size)
        if sequential:
            ing.sync()
    ing.sync()
    snap, modes, pats = st.read(len(chunks))
    alarms = [int(a) for a in st.read_alarms(len(chunks))] if extra and extra.get("alarm_pct") else None
    got = outs.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    st.close()
    ing.close()
    return got, snap, modes, pats, alarms


@pytest.mark.parametrize("n_hip,lag,W,sequential,source", [(1, 0, 1, True, "pinned"), (1, 0, 1, False, "pinned"),
                                                           (3, 2, 3, False, "pinned"), (8, 0, 1, False, "pinned"),
                                                           (8, 5, 2, False, "pinned"), (2, 1, 1, False, "pageable")])
def test_ingest_matches_oracle(hm, n_hip, lag, W, sequential, source):
    chunks = chunks_mixed(500 + n_hip * 10 + lag, 40, 300_000)
    ref = O.stream_reference(chunks, W=W, theta_pct=45, S=960, rmax=8, lag=lag)
    got, snap, modes, pats, _ = run(hm, chunks, n_hip, W, 45, 960, 8, lag, sequential, source)
    assert np.array_equal(got, ref["hists"].astype(np.int64))
    assert [int(x) for x in snap.acc] == ref["acc"]
    assert [int(x) for x in snap.mw] == ref["mw"]
    assert [int(m) for m in modes] == ref["modes"]
    assert [list(map(int, p)) for p in pats] == ref["patterns"]
    d = hm.diag()
    assert d.invalid_patterns == 0 and d.wait_timeouts == 0 and d.merge_timeouts == 0


@pytest.mark.parametrize("W,alarm_pct,criterion,kappa", [(1, 10, 1, 5), (4, 5, 2, 20)])
def test_ingest_with_detection_and_criterion(hm, W, alarm_pct, criterion, kappa):
    # host-fed streams with change detection and the alternative switching criterion on
    chunks = chunks_mixed(800 + W, 48, 200_000)
    ref = O.stream_reference(chunks, W=W, theta_pct=45, S=960, rmax=8, lag=1, alarm_pct=alarm_pct,
                             criterion=criterion, kappa_pct=kappa)
    got, snap, modes, pats, alarms = run(hm, chunks, 4, W, 45, 960, 8, 1,
                                         extra={"alarm_pct": alarm_pct, "criterion": criterion, "kappa_pct": kappa})
    assert np.array_equal(got, ref["hists"].astype(np.int64))
    assert [int(x) for x in snap.acc] == ref["acc"]
    assert [int(x) for x in snap.mw] == ref["mw"]
    assert [int(m) for m in modes] == ref["modes"]
    assert [list(map(int, p)) for p in pats] == ref["patterns"]
    assert alarms == ref["alarms"]
    assert int(snap.alarms) == sum(ref["alarms"])
    d = hm.diag()
    assert d.invalid_patterns == 0 and d.wait_timeouts == 0 and d.merge_timeouts == 0


def test_ingest_full_size_single_stream(hm):
    # the 66 x 4 MiB stream from pinned host memory over 16 HIP streams, the bench's settings
    chunks = G.stream_chunks(4 << 20)
    hists = [O.hist(c) for c in chunks]
    ref = O.stream_reference(None, W=1, theta_pct=0, S=8192, rmax=32, lag=31, hists=hists)
    got, snap, modes, pats, _ = run(hm, chunks, 16, 1, 0, 8192, 32, 31)
    assert np.array_equal(got, ref["hists"].astype(np.int64))
    assert [int(m) for m in modes] == ref["modes"]
    assert [int(x) for x in snap.acc] == ref["acc"]


def test_ingest_errors(hm):
    ing = hm.Ingest(n_hip_streams=2, slot_bytes=4096)
    st = hm.Stream()
    with pytest.raises(hm.HistError) as e:
        ing.push(st, np.zeros(5000, np.uint8))
    assert e.value.status == hm.EINVAL
    with pytest.raises(hm.HistError):
        ing.push(st, 0, n=16)
    ing.push(st, np.zeros(0, np.uint8))    # an empty chunk is a chunk
    ing.sync()
    snap, _, _ = st.read(0)
    assert int(snap.chunks) == 1
    st.close()
    ing.close()
