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
