"""hist_u8_noalloc, the entry point for callers that cannot allocate device memory, against
hist_u8 and the oracle: two calls in a row (the second on a smaller input, so it reuses the
fixed scratch array the first left behind), every kind of counting table, empty and ragged
inputs, and replays of a captured HIP graph.  Counts are integers: the bar is bit-exact."""

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _u32(t):
    return t.cpu().numpy().astype(np.int64) & 0xFFFFFFFF


def _modes(hm):
    return [("auto", hm.MODE_AUTO, None), ("wavehist", hm.MODE_WAVEHIST, None),
            ("waveagg", hm.MODE_WAVEAGG, None), ("ahist-identity", hm.MODE_AHIST, None),
            ("ahist-paper960", hm.MODE_AHIST, hm.pattern_init(hm.PAT_PAPER960))]


def test_two_calls_match_hist_u8(hm):
    g = np.random.default_rng(20)
    host = g.integers(0, 256, size=(16 << 20) + 64, dtype=np.uint8)
    host[5:(1 << 18)] = 77                        # a degenerate stretch
    d = torch.from_numpy(host).cuda()
    base = int(d.data_ptr())
    # first a large ragged input (every workgroup, the most partial copies), then a smaller one
    for name, mode, pat in _modes(hm):
        for n1, off1, n2, off2 in (((16 << 20) + 5, 3, 100003, 1), ((1 << 20) + 13, 0, 4097, 7)):
            print("case", name, n1, off1, n2, off2, flush=True)
            outs = []
            for n, off in ((n1, off1), (n2, off2)):
                a = torch.full((256,), -1, dtype=torch.int32, device="cuda")
                b = torch.full((256,), -1, dtype=torch.int32, device="cuda")
                hm.hist_u8_noalloc(base + off, a, mode=mode, pattern=pat, n=n)
                hm.hist_u8(base + off, b, mode=mode, pattern=pat, n=n)
                outs.append((a, b, host[off:off + n]))
            torch.cuda.synchronize()
            for a, b, ref in outs:
                exp = O.hist(ref).astype(np.int64)
                assert np.array_equal(_u32(a), _u32(b)), name
                assert np.array_equal(_u32(a), exp), name


def test_empty_and_tiny_inputs(hm):
    d = torch.arange(64, dtype=torch.uint8, device="cuda")
    for n in (0, 1, 15, 17, 64):
        out = torch.full((256,), -1, dtype=torch.int32, device="cuda")
        hm.hist_u8_noalloc(d, out, n=n)
        torch.cuda.synchronize()
        exp = np.zeros(256, dtype=np.int64)
        exp[:n] = 1
        assert np.array_equal(_u32(out), exp), n


def test_argument_errors(hm):
    out = torch.zeros(256, dtype=torch.int32, device="cuda")
    lib = hm.load()
    assert lib.hist_u8_noalloc(None, 10, int(out.data_ptr()), hm.MODE_AUTO, None, 0) == hm.EINVAL
    assert lib.hist_u8_noalloc(None, 0, None, hm.MODE_AUTO, None, 0) == hm.EINVAL
    assert lib.hist_u8_noalloc(int(out.data_ptr()), 16, int(out.data_ptr()), 9, None, 0) == hm.EINVAL
    assert lib.hist_u8_noalloc(int(out.data_ptr()), 1 << 32, int(out.data_ptr()), hm.MODE_AUTO, None, 0) \
        == hm.EOVERFLOW


def test_graph_replays(hm):
    """Captured once into a HIP graph (kernel nodes only) and replayed over changing bytes,
    with eager work and synchronisation between the replays: every replay is exact."""
    g = np.random.default_rng(21)
    n = (3 << 20) + 11
    d = torch.from_numpy(g.integers(0, 256, size=n, dtype=np.uint8)).cuda()
    out = torch.zeros(256, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    hm.hist_u8_noalloc(d, out, stream=s)          # set-up happens outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        hm.hist_u8_noalloc(d, out, stream=s)
    for rep in range(4):
        fresh = g.integers(0, 256, size=n, dtype=np.uint8)
        if rep == 2:
            fresh[:] = 9
        d.copy_(torch.from_numpy(fresh))
        out.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(_u32(out), O.hist(fresh).astype(np.int64)), rep
    del graph
