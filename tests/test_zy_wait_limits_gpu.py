"""Bounded decision waits that give up, forced from the host (one poll per wait).

The library counts every wait that gives up in process-wide diagnostics (hist_diag_read),
which the other GPU tests require to stay zero; this file's name sorts after theirs, so the
counts it leaves behind come last (only the no-allocation entry point's test, which reads no
diagnostics, runs after it).
"""

import numpy as np
import pytest

from oracle import oracle as O
import synthgen as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("W, alarm", [(32, 0), (5, 4), (1, 0)])
def test_decision_waits_that_give_up(hm, W, alarm):
    # Force the bounded decision waits to give up from the host (one poll each): chunks then
    # run the per-wavefront kernel without their decision, and still write their histograms
    # into the stream's ring.  Counts, the Accumulator, the moving window, the chunk count
    # and the change-detection alarms must stay exact (the ring holds every chunk two
    # launches in flight can produce, whatever waits), and the stream read must report the
    # timeouts as HIST_ETIMEDOUT.
    chunks = G.stream_chunks(256 << 10)
    hists = [O.hist(c) for c in chunks] * 3
    theta, S, rmax, lag = 45, 960, 8, 0
    ref = O.stream_reference(None, W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, hists=hists, alarm_pct=alarm)
    d = dev(np.concatenate(chunks))
    base = int(d.data_ptr())
    bufs = [(base + k * (256 << 10), 256 << 10) for k in range(len(chunks))]
    outs = [torch.full((len(chunks), 256), -1, dtype=torch.int32, device="cuda") for _ in range(3)]
    d0 = int(hm.diag().wait_timeouts)
    hm.set_wait_limits(decision_polls=1)
    try:
        st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=len(hists), alarm_pct=alarm)
        torch.cuda.synchronize()
        hs = [torch.cuda.Stream(), torch.cuda.Stream()]
        for r in range(3):
            st.push_many(bufs, d_out=outs[r], stream=hs[r & 1])
        with pytest.raises(hm.HistError) as e:
            st.read(0, stream=hs[0])
        assert e.value.status == hm.ETIMEDOUT
        snap, _, _ = st.read(0, stream=hs[0], allow_timeouts=True)
        al = st.read_alarms(len(hists), stream=hs[0]) if alarm else None
        torch.cuda.synchronize()
        st.close()
    finally:
        hm.set_wait_limits(0, 0)
    got = np.concatenate([o.cpu().numpy().astype(np.int64) & 0xFFFFFFFF for o in outs])
    assert np.array_equal(got, ref["hists"].astype(np.int64))
    assert [int(x) for x in snap.acc] == ref["acc"]
    assert int(snap.chunks) == len(hists)
    assert snap.wait_timeouts > 0 and snap.merge_timeouts == 0
    assert int(hm.diag().wait_timeouts) - d0 == snap.wait_timeouts
    if W > 1:
        assert [int(x) for x in snap.mw] == ref["mw"]
    if alarm:
        assert [int(x) for x in al] == ref["alarms"]
        assert int(snap.alarms) == sum(ref["alarms"])
