"""Maximum sizes (Sec. III.A: exact counts).

The largest hist_u8 input is 2^32 - 1 bytes, where a single bin can hold the largest 32-bit
count, and hist_u8_u64 takes inputs beyond 2^32 bytes (accumulated in pieces).  Inputs this
large are checked against closed forms rather than a CPU pass: a ramp of bytes i mod 256
(value v occurs floor((n - 1 - v) / 256) + 1 times) and a buffer of one value.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N32 = (1 << 32) - 1


def u32(out):
    return (out.cpu().numpy().astype(np.int64) & 0xFFFFFFFF).tolist()


def test_largest_input_ramp(hm):
    d = torch.arange(256, dtype=torch.uint8, device="cuda").repeat(1 << 24)   # 4 GiB of i mod 256
    out = torch.full((256,), -1, dtype=torch.int32, device="cuda")
    hm.hist_u8(d, out, n=N32)
    assert u32(out) == [(N32 - 1 - v) // 256 + 1 for v in range(256)]
    del d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mode", ["auto", "wavehist"])
def test_one_value_fills_a_32bit_bin(hm, mode):
    # 2^32 - 1 bytes of one value: its bin ends at the largest 32-bit count, through the
    # partial copies and the finalizer's sum (the degenerate case the per-wavefront kernel
    # serialises on, at its largest)
    d = torch.full((N32,), 255, dtype=torch.uint8, device="cuda")
    out = torch.full((256,), -1, dtype=torch.int32, device="cuda")
    hm.hist_u8(d, out, mode=hm.MODE_AUTO if mode == "auto" else hm.MODE_WAVEHIST)
    want = [0] * 256
    want[255] = N32
    assert u32(out) == want
    del d
    torch.cuda.empty_cache()


def test_u64_beyond_32_bits(hm):
    n = (1 << 32) + 12345
    d = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    acc = torch.zeros(256, dtype=torch.int64, device="cuda")
    hm.hist_u8_u64(d, acc)
    hm.hist_u8_u64(d, acc, n=12345)   # accumulates
    a = acc.cpu().numpy()
    assert int(a[7]) == n + 12345 and int(a.sum()) == n + 12345
    del d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("W,theta,S,rmax", [(2, 0, 8192, 32), (1, 45, 960, 8)])
def test_largest_stream_chunk(hm, W, theta, S, rmax):
    # a stream chunk of 2^32 - 1 bytes (a ramp) then one of 1000 bytes of value 9: per-chunk
    # histograms, the Accumulator and the window (W = 2: both chunks) against closed forms.
    # The uniform switch runs the launch on equal shares (the window is summed on read);
    # theta 45 at lag 0 runs it on one slice per workgroup of each chunk.
    d = torch.arange(256, dtype=torch.uint8, device="cuda").repeat(1 << 24)
    small = torch.full((1000,), 9, dtype=torch.uint8, device="cuda")
    ramp = [(N32 - 1 - v) // 256 + 1 for v in range(256)]
    nine = [1000 if v == 9 else 0 for v in range(256)]
    st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=0, trace_cap=2)
    outs = torch.full((2, 256), -1, dtype=torch.int32, device="cuda")
    st.push_many([(int(d.data_ptr()), N32), (int(small.data_ptr()), 1000)], d_out=outs)
    snap, _, _ = st.read(2)
    assert u32(outs[0]) == ramp and u32(outs[1]) == nine
    total = [a + b for a, b in zip(ramp, nine)]
    assert [int(x) for x in snap.acc] == total
    assert [int(x) for x in snap.mw] == (total if W == 2 else nine)
    assert int(snap.chunks) == 2
    st.close()
    del d
    torch.cuda.empty_cache()
