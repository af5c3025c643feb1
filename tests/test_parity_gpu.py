"""GPU parity of hist_u8 / hist_u8_u64 against the oracle: every mode and pattern, ragged sizes,
every pointer offset 0..15, the paper's input types, and full-size inputs.  Counts are
integers: the bar is bit-exact."""

import numpy as np
import pytest

from oracle import oracle as O
import synthgen as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_u8(hm, d_in, n, mode, pattern=None, offset=0):
    out = torch.full((256,), -1, dtype=torch.int32, device="cuda")   # overwritten, not accumulated
    hm.hist_u8(int(d_in.data_ptr()) + offset, out, mode=mode, pattern=pattern, n=n)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.int64) & 0xFFFFFFFF


def patterns(hm):
    """(name, mode, host pattern) for every kernel variant."""
    rnd = np.random.default_rng(7)
    out = [("auto", hm.MODE_AUTO, None), ("wavehist", hm.MODE_WAVEHIST, None), ("waveagg", hm.MODE_WAVEAGG, None),
           ("ahist-identity", hm.MODE_AHIST, None),
           ("ahist-paper960", hm.MODE_AHIST, hm.pattern_init(hm.PAT_PAPER960)),
           ("ahist-flat2", hm.MODE_AHIST, hm.pattern_init(hm.PAT_FLAT, 0, 2)),
           ("ahist-flat32", hm.MODE_AHIST, hm.pattern_init(hm.PAT_FLAT, 0, 32)),
           ("ahist-flat64", hm.MODE_AHIST, hm.pattern_init(hm.PAT_FLAT, 0, 64))]
    # rule-P patterns (from the oracle) of skewed histograms: non-uniform, buddy-aligned
    for k, (S, rmax) in enumerate([(960, 8), (2048, 32), (4000, 64)]):
        h = rnd.integers(0, 1000, 256) ** 3
        w = O.rule_p(h.tolist(), S, rmax)
        out.append(("ahist-ruleP-%d-%d" % (S, rmax), hm.MODE_AHIST, hm.Pattern.from_words(w, S, rmax)))
    # a valid but unaligned, shuffled layout
    r = [1 << int(x) for x in rnd.integers(0, 4, 256)]
    order = rnd.permutation(256)
    w = O.pattern_from_r(r, order)
    out.append(("ahist-shuffled", hm.MODE_AHIST, hm.Pattern.from_words(w, sum(r), 8)))
    return out


SIZES = [0, 1, 15, 16, 17, 31, 33, 1023, 1024, 4097, 65536 + 13, (1 << 20) + 13, (16 << 20) + 5]


def test_every_mode_every_size(hm):
    g = np.random.default_rng(11)
    host = g.integers(0, 256, size=(16 << 20) + 64, dtype=np.uint8)
    host[: 1 << 16] = 200           # a degenerate stretch at the front
    d = dev(host)
    for name, mode, pat in patterns(hm):
        for n in SIZES:
            for off in (0, 3):
                print("case", name, n, off, flush=True)
                got = run_u8(hm, d, n, mode, pat, off)
                exp = O.hist(host[off:off + n]).astype(np.int64)
                assert np.array_equal(got, exp), (name, n, off)


def test_every_offset(hm):
    g = np.random.default_rng(12)
    host = G.clipped_normal_bytes((1 << 20) + 64, 90.0, 3.0, g)
    d = dev(host)
    for name, mode, pat in patterns(hm)[:7]:
        for off in range(16):
            n = (1 << 20) + 1 - off
            got = run_u8(hm, d, n, mode, pat, off)
            assert np.array_equal(got, O.hist(host[off:off + n]).astype(np.int64)), (name, off)


@pytest.mark.parametrize("kind", G.TABLE2_KINDS)
def test_table2_inputs_full_size(hm, kind):
    # the paper's 8192 x 8192 slice, each input type, all modes
    host = G.table2_input(kind)
    exp = O.hist(host).astype(np.int64)
    d = dev(host)
    for name, mode, pat in patterns(hm)[:8]:
        got = run_u8(hm, d, host.size, mode, pat)
        assert np.array_equal(got, exp), (kind, name)
        assert int(got.sum()) == host.size


def test_image_1mib(hm):
    host = G.image_1mib()
    exp = O.hist(host).astype(np.int64)
    d = dev(host)
    for name, mode, pat in patterns(hm):
        assert np.array_equal(run_u8(hm, d, host.size, mode, pat), exp), name


def test_u64_accumulates(hm):
    g = np.random.default_rng(13)
    host = g.integers(0, 256, size=3 << 20, dtype=np.uint8)
    d = dev(host)
    acc = torch.zeros(256, dtype=torch.int64, device="cuda")
    for mode in (hm.MODE_AUTO, hm.MODE_WAVEHIST, hm.MODE_AHIST, hm.MODE_WAVEAGG):
        hm.hist_u8_u64(d, acc, mode=mode)
    hm.hist_u8_u64(d, acc, mode=hm.MODE_AUTO, n=0)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), 4 * O.hist(host).astype(np.int64))


def test_repeat_is_deterministic(hm):
    host = G.table2_input("xray", 8 << 20)
    d = dev(host)
    exp = O.hist(host).astype(np.int64)
    for _ in range(20):
        assert np.array_equal(run_u8(hm, d, host.size, hm.MODE_AUTO), exp)


def test_argument_errors_on_device(hm):
    out = torch.zeros(256, dtype=torch.int32, device="cuda")
    with pytest.raises(hm.HistError) as e:
        hm.hist_u8(0, out, n=10)
    assert e.value.status == hm.EINVAL
    with pytest.raises(hm.HistError) as e:
        hm.hist_u8(int(out.data_ptr()), out, n=1 << 32)   # a raw address: the library's own check
    assert e.value.status == hm.EOVERFLOW
    bad = hm.pattern_init(hm.PAT_IDENTITY)
    bad.word[1] = bad.word[0]
    with pytest.raises(hm.HistError) as e:
        hm.hist_u8(out, out, mode=hm.MODE_AHIST, pattern=bad, n=16)
    assert e.value.status == hm.EINVAL
    with pytest.raises(hm.HistError) as e:
        hm.hist_u8(out, out, mode=7, n=16)
    assert e.value.status == hm.EINVAL


def test_pattern_update_matches_oracle_rule(hm):
    rnd = np.random.default_rng(14)
    cases = [np.zeros(256, np.int64), np.full(256, 1000, np.int64)]
    one = np.zeros(256, np.int64)
    one[127] = 4 << 20
    cases.append(one)
    two = np.zeros(256, np.int64)
    two[0] = two[255] = 1 << 21
    cases.append(two)
    for _ in range(20):
        cases.append(rnd.integers(0, 1 << rnd.integers(1, 40), 256))
    cases.append(np.full(256, (1 << 55) // 256, np.int64))
    for h in cases:
        for S, rmax in [(960, 8), (256, 64), (300, 16), (8192, 32), (8191, 32), (16384, 64), (5000, 64)]:
            dh = torch.from_numpy(h.astype(np.int64)).cuda()
            dp = torch.zeros(258, dtype=torch.int32, device="cuda")
            hm.pattern_update(dh, S, rmax, dp)
            torch.cuda.synchronize()
            words = (dp.cpu().numpy().astype(np.int64) & 0xFFFFFFFF).tolist()
            assert words[:256] == O.rule_p(h.tolist(), S, rmax), (S, rmax)
            assert words[256] == S and words[257] == rmax


def test_read_probe_sums_every_word(hm):
    # the read-roofline probe reads each 16-byte vector once: its sum of uint32 words is exact
    g = np.random.default_rng(15)
    for n in (16, 4096, (1 << 20) + 16 * 7, 3 << 22):
        host = g.integers(0, 256, size=n, dtype=np.uint8)
        d = dev(host)
        acc = torch.zeros(1, dtype=torch.int64, device="cuda")
        hm.read_probe(d, acc)
        hm.read_probe(d, acc, workgroups=3)
        torch.cuda.synchronize()
        exp = 2 * int(host.view(np.uint32).astype(np.uint64).sum())
        assert int(acc.item()) == exp, n
    with pytest.raises(hm.HistError):
        hm.read_probe(d, acc, n=15)
