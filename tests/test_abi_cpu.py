"""Host-only checks of the C ABI (no GPU calls): the library loads, exports every symbol the
header declares, the binding declares exactly those, and argument errors that are decided
before any device work come back synchronously with the documented status."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "histmi.h")


@pytest.fixture(scope="module")
def hm():
    import paper_1011_0235_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1011_0235_amd import build
        build.build()
    m.load()
    return m


def header_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:hist_status_t|const char \*)\s*(hist_[a-z0-9_]+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    syms = header_symbols()
    for must in ("hist_u8", "hist_u8_u64", "hist_pattern_update", "hist_batch", "hist_server_create",
                 "hist_server_submit", "hist_stream_push", "hist_strerror"):
        assert must in syms


def test_library_exports_every_declared_symbol(hm):
    lib = ctypes.CDLL(hm.LIB_PATH)
    for name in header_symbols():
        assert hasattr(lib, name), name
    assert sorted(hm.declared_symbols()) == header_symbols()


def test_timeline_build_exports_its_calls(hm):
    # the diagnostic twin (kernel compiled with HISTMI_TIMELINE) exports the same ABI plus
    # the three calls include/histmi_timeline.h declares; the default library does not
    tl_path = os.path.join(os.path.dirname(hm.LIB_PATH), "libhistmi_timeline.so")
    assert os.path.exists(tl_path)
    tl = ctypes.CDLL(tl_path)
    text = open(os.path.join(ROOT, "include", "histmi_timeline.h")).read()
    calls = sorted(set(re.findall(r"^int (hist_timeline_[a-z_]+)\(", text, re.M)))
    assert calls == ["hist_timeline_read", "hist_timeline_reset", "hist_timeline_shape"]
    for name in calls + header_symbols():
        assert hasattr(tl, name), name
    lib = ctypes.CDLL(hm.LIB_PATH)
    for name in calls:
        assert not hasattr(lib, name), name


def test_strerror(hm):
    for st in (hm.OK, hm.EINVAL, hm.ENOMEM, hm.EOVERFLOW, hm.EBUSY, hm.EDEVICE, hm.ENOTSUP, hm.ETIMEDOUT,
               hm.ECANCELED):
        assert hm.strerror(st) and hm.strerror(st) != "unknown status"
    assert hm.strerror(-99) == "unknown status"


def test_pattern_presets_match_the_oracle(hm):
    assert hm.pattern_init(hm.PAT_IDENTITY).words() == O.pattern_identity()
    p = hm.pattern_init(hm.PAT_PAPER960)
    assert p.words() == O.pattern_paper960() and p.total_S == 960 and p.rmax == 8
    for r in (1, 2, 8, 32, 64):
        p = hm.pattern_init(hm.PAT_FLAT, 0, r)
        assert p.words() == O.pattern_flat(r) and p.total_S == 256 * r
    with pytest.raises(hm.HistError):
        hm.pattern_init(hm.PAT_FLAT, 0, 3)
    with pytest.raises(hm.HistError):
        hm.pattern_init(7)


@pytest.mark.parametrize("seed", range(30))
def test_pattern_validate_agrees_with_oracle(hm, seed):
    rnd = np.random.default_rng(seed)
    S = int(rnd.choice([256, 300, 960, 4096, 16384, 20000]))
    rmax = int(rnd.choice([1, 2, 8, 32, 64, 128]))
    kind = seed % 3
    if kind == 0:
        words = O.rule_p(rnd.integers(0, 1000, 256).tolist(), max(256, min(S, 16384)), min(rmax, 64))
    elif kind == 1:
        words = [int(x) for x in rnd.integers(0, 1 << 20, 256)]
    else:
        words = O.pattern_identity()
        i, j = rnd.integers(0, 256, 2)
        words[int(i)] = words[int(j)]
    p = hm.Pattern.from_words(words, S, rmax)
    ok = (hm.pattern_validate(p) == hm.OK)
    expect = (rmax <= 64 and S <= 16384 and O.pattern_valid(words, S, rmax))
    assert ok == expect


def test_synchronous_argument_errors(hm):
    lib = hm.load()
    # NULL input with n > 0, NULL output, bad mode, n too large: refused before any device work
    out = ctypes.c_void_p(0x1000)
    assert lib.hist_u8(None, 10, out, 0, None, None) == hm.EINVAL
    assert lib.hist_u8(ctypes.c_void_p(0x1000), 10, None, 0, None, None) == hm.EINVAL
    assert lib.hist_u8(ctypes.c_void_p(0x1000), 10, out, 9, None, None) == hm.EINVAL
    assert lib.hist_u8(ctypes.c_void_p(0x1000), 1 << 32, out, 0, None, None) == hm.EOVERFLOW
    bad = hm.pattern_init(hm.PAT_IDENTITY)
    bad.word[5] = bad.word[6]
    assert lib.hist_u8(ctypes.c_void_p(0x1000), 10, out, hm.MODE_AHIST, ctypes.byref(bad), None) == hm.EINVAL
    assert lib.hist_u8_u64(None, 10, out, 0, None, None) == hm.EINVAL
    assert lib.hist_pattern_update(None, 960, 8, out, None) == hm.EINVAL
    assert lib.hist_pattern_update(out, 255, 8, out, None) == hm.EINVAL
    assert lib.hist_pattern_update(out, 960, 3, out, None) == hm.EINVAL
    assert lib.hist_read_probe(None, 16, out, 0, None) == hm.EINVAL
    assert lib.hist_read_probe(ctypes.c_void_p(0x1000), 17, out, 0, None) == hm.EINVAL
    assert lib.hist_read_probe(ctypes.c_void_p(0x1008), 16, out, 0, None) == hm.EINVAL
    assert lib.hist_read_probe(ctypes.c_void_p(0x1000), 16, out, 70000, None) == hm.EINVAL
    assert lib.hist_read_probe(ctypes.c_void_p(0x1000), 0, None, 0, None) == hm.OK


def test_stream_and_server_config_errors(hm):
    lib = hm.load()
    h = ctypes.c_void_p()
    for cfg in (hm._lib.StreamConfig(0, 45, 960, 8, 0, 1), hm._lib.StreamConfig(1, 101, 960, 8, 0, 1),
                hm._lib.StreamConfig(1, 45, 100, 8, 0, 1), hm._lib.StreamConfig(1, 45, 960, 6, 0, 1),
                hm._lib.StreamConfig(1, 45, 20000, 8, 0, 1), hm._lib.StreamConfig(32, 45, 960, 8, 0, 1, 101),
                hm._lib.StreamConfig(4, 45, 960, 8, 0, 1, 0, 3, 10), hm._lib.StreamConfig(4, 45, 960, 8, 0, 1, 0, 1, 101)):
        assert lib.hist_stream_create(ctypes.byref(h), ctypes.byref(cfg)) == hm.EINVAL
    assert lib.hist_stream_read_alarms(None, None, 0, None) == hm.EINVAL
    for cfg in (hm._lib.ServerConfig(0, 4, 4, 1, 4, 0, 45, 960, 8), hm._lib.ServerConfig(1 << 20, 0, 4, 1, 4, 0, 45, 960, 8),
                hm._lib.ServerConfig(1 << 20, 4, 4, 17, 4, 0, 45, 960, 8),
                hm._lib.ServerConfig(1 << 20, 4, 4, 1, 4, 5, 45, 960, 8),
                hm._lib.ServerConfig(1 << 20, 4, 4, 1, 4, 0, 45, 960, 8, 10000001)):
        assert lib.hist_server_create(ctypes.byref(h), ctypes.byref(cfg)) == hm.EINVAL
    for cfg in (hm._lib.IngestConfig(0, 1 << 20), hm._lib.IngestConfig(257, 1 << 20), hm._lib.IngestConfig(4, 0),
                hm._lib.IngestConfig(4, 1 << 33)):
        assert lib.hist_ingest_create(ctypes.byref(h), ctypes.byref(cfg)) == hm.EINVAL
    assert lib.hist_ingest_push(None, None, None, 0, 0, None) == hm.EINVAL
    assert lib.hist_ingest_sync(None) == hm.EINVAL
    assert lib.hist_stream_push(None, None, 0, 0, None, None) == hm.EINVAL
    assert lib.hist_server_submit(None, 0, None, 0, None, None) == hm.EINVAL


def test_tuning_table(hm):
    for fam in (1, hm.TUNE_STREAM, hm.TUNE_STREAM_KNOWN):
        old = hm.tune_get(fam)
        hm.tune_set(fam, blocks_per_cu=3, tile_kib=128, merge_copies=8, tiles_per_wg=5)
        t = hm.tune_get(fam)
        assert (t.blocks_per_cu, t.tile_kib, t.merge_copies, t.tiles_per_wg) == (3, 128, 8, 5)
        hm.tune_set(fam, old.blocks_per_cu, old.tile_kib, old.merge_copies, old.tiles_per_wg)
    with pytest.raises(hm.HistError):
        hm.tune_set(1, tile_kib=17)
    with pytest.raises(hm.HistError):
        hm.tune_set(1, merge_copies=3)
    with pytest.raises(hm.HistError):
        hm.tune_set(1, tiles_per_wg=65)
    with pytest.raises(hm.HistError):
        hm.tune_set(6, blocks_per_cu=1)


def test_struct_layouts_match_binding(hm, tmp_path):
    # every struct of the C ABI, compiled by the host compiler from include/histmi.h, has the
    # size and field offsets the binding's ctypes mirror assumes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not installed")
    L = hm._lib
    pairs = {"hist_pattern_t": L.Pattern, "hist_device_info_t": L.DeviceInfo,
             "hist_stream_config_t": L.StreamConfig, "hist_ingest_config_t": L.IngestConfig,
             "hist_stream_snapshot_t": L.StreamSnapshot, "hist_diag_t": L.Diag, "hist_tune_t": L.Tune,
             "hist_server_config_t": L.ServerConfig, "hist_server_result_t": L.ServerResult,
             "hist_server_stats_t": L.ServerStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "histmi.h"', 'int main(void) {']
    for cname, cls in pairs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines.append('return 0; }')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, cls in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert got[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])


def test_buffer_marshalling_forms():
    # the binding's buffer lists: pairs, an (n, 2) array and the per-item path agree
    from paper_1011_0235_amd import _lib as L

    class Buf:   # what the binding reads of a device tensor
        def __init__(self, addr, n):
            self.addr, self.n = addr, n

        def data_ptr(self):
            return self.addr

        def numel(self):
            return self.n

        def element_size(self):
            return 1

    pairs = [((1 << 40) + 4096 * i, 1000 + i) for i in range(300)] + [(0, 0)]
    p1, s1 = L._ptr_arrays(pairs)
    p2, s2 = L._ptr_arrays(np.array(pairs, dtype=np.int64))
    p3, s3 = L._ptr_arrays([Buf(a, n) if i % 2 else (a, n) for i, (a, n) in enumerate(pairs)])
    for p, q in ((p1, s1), (p2, s2), (p3, s3)):
        assert p.dtype == np.uint64 and q.dtype == np.uint64 and p.flags.c_contiguous and q.flags.c_contiguous
    assert np.array_equal(p1, p2) and np.array_equal(s1, s2)
    assert np.array_equal(p1, p3) and np.array_equal(s1, s3)
    assert [int(x) for x in p1[:3]] == [1 << 40, (1 << 40) + 4096, (1 << 40) + 8192]
    assert int(s1[-1]) == 0 and int(p1[-1]) == 0 and len(p1) == 301
    for bad in (np.zeros((3, 3), dtype=np.int64), np.zeros((3, 2), dtype=np.float64), np.array([[-1, 5]])):
        with pytest.raises(ValueError):
            L._ptr_arrays(bad)


def test_binding_refuses_sizes_beyond_the_tensors(hm):
    # an explicit n beyond the input tensor's bytes would make the kernel read past the
    # allocation, and a short or wrongly typed output would be written past its end: the
    # binding refuses both before anything reaches the library
    import torch
    x = torch.zeros(100, dtype=torch.uint8)
    out = torch.zeros(256, dtype=torch.int32)
    with pytest.raises(ValueError):
        hm.hist_u8(x, out, n=101)
    with pytest.raises(ValueError):
        hm.hist_u8(x, torch.zeros(255, dtype=torch.int32))
    with pytest.raises(ValueError):
        hm.hist_u8(x, torch.zeros(256, dtype=torch.int64))
    with pytest.raises(ValueError):
        hm.hist_u8(x, torch.zeros(512, dtype=torch.int32)[::2])
    with pytest.raises(ValueError):
        hm.hist_u8_u64(x, torch.zeros(256, dtype=torch.int32))
    with pytest.raises(ValueError):
        hm.read_probe(x, torch.zeros(1, dtype=torch.int64), n=112)
    with pytest.raises(ValueError):
        hm.hist_batch([x, x], torch.zeros((1, 256), dtype=torch.int32))
    with pytest.raises(ValueError):
        hm.hist_u8(12345, out)   # a raw address needs n
