"""GPU parity of batched histograms (many slices in one asynchronous call, Sec. III.B):
every output against the oracle, uneven and empty images, byte-packed (unaligned) arenas,
all modes, and HIP-graph replays with eager work between them."""

import numpy as np
import pytest

from oracle import oracle as O
import synthgen as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_batch(hm, arena, offs, sizes, mode=0, pattern=None):
    d = dev(arena)
    base = int(d.data_ptr())
    bufs = [(base + int(o), int(n)) for o, n in zip(offs, sizes)]
    out = torch.full((len(bufs), 256), -1, dtype=torch.int32, device="cuda")
    hm.hist_batch(bufs, out, mode=mode, pattern=pattern)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.int64) & 0xFFFFFFFF


@pytest.mark.parametrize("align", [256, 1])
def test_batch_image_shapes(hm, align):
    specs = G.batch_specs(96, 64, 1024)          # the batch's distributions, sides up to 1024
    arena, offs, sizes = G.batch_arena(specs, align=align)
    exp = O.hist_many(arena, offs, sizes).astype(np.int64)
    for mode, pat in ((hm.MODE_AUTO, None), (hm.MODE_WAVEHIST, None), (hm.MODE_AHIST, None),
                      (hm.MODE_AHIST, hm.pattern_init(hm.PAT_PAPER960))):
        got = run_batch(hm, arena, offs, sizes, mode, pat)
        assert np.array_equal(got, exp), (align, mode)


def test_batch_uneven_with_empty_and_large(hm):
    g = np.random.default_rng(3)
    sizes = [0, 1, 15, 16, 17, 4096, 0, (16 << 20) + 3, 1 << 20, 777, 0, 65536 * 3 + 5]
    offs, pos = [], 0
    for n in sizes:
        pos += int(g.integers(0, 16))
        offs.append(pos)
        pos += n
    arena = g.integers(0, 256, size=pos + 16, dtype=np.uint8)
    arena[offs[7]:offs[7] + (1 << 20)] = 9          # a degenerate stretch inside the big image
    exp = O.hist_many(arena, offs, sizes).astype(np.int64)
    for mode in (hm.MODE_AUTO, hm.MODE_WAVEHIST, hm.MODE_AHIST, hm.MODE_WAVEAGG):
        assert np.array_equal(run_batch(hm, arena, offs, sizes, mode), exp), mode


def test_batch_many_tiny(hm):
    g = np.random.default_rng(4)
    sizes = g.integers(0, 300, size=3000)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    arena = g.integers(0, 256, size=int(sizes.sum()) + 1, dtype=np.uint8)
    exp = O.hist_many(arena, offs, sizes).astype(np.int64)
    assert np.array_equal(run_batch(hm, arena, offs, sizes), exp)


def test_batch_graph_replays(hm):
    specs = G.batch_specs(64, 64, 512)
    arena, offs, sizes = G.batch_arena(specs, align=256)
    d = dev(arena)
    base = int(d.data_ptr())
    bufs = [(base + int(o), int(n)) for o, n in zip(offs, sizes)]
    out = torch.full((len(bufs), 256), -1, dtype=torch.int32, device="cuda")
    graph = hm.BatchGraph(bufs, out, mode=hm.MODE_AUTO)
    exp = O.hist_many(arena, offs, sizes).astype(np.int64)
    for rep in range(5):
        out.fill_(-1)
        graph.launch()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().astype(np.int64), exp), rep
        # eager work between replays on the same buffers (also changes them, then restores)
        tmp = torch.zeros(256, dtype=torch.int32, device="cuda")
        hm.hist_u8(d, tmp)
        d.add_(1)
        graph.launch()
        torch.cuda.synchronize()
        shifted = O.hist_many((arena + 1).astype(np.uint8), offs, sizes).astype(np.int64)
        assert np.array_equal(out.cpu().numpy().astype(np.int64), shifted), rep
        d.sub_(1)
    graph.close()


def batch_arena_on_device(specs, seed):
    """The 4096-image batch generated on the device: each image uniform, a clipped
    Normal(mu, sigma) or a 90 % spike at one value (the rest uniform), at 256-byte aligned
    offsets of one arena."""
    sizes = np.array([s.size for s in specs], dtype=np.int64)
    offs = np.zeros_like(sizes)
    offs[1:] = np.cumsum((sizes + 255) // 256 * 256)[:-1]
    total = int(offs[-1] + sizes[-1])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    arena = torch.randint(0, 256, (total,), dtype=torch.uint8, device="cuda", generator=gen)
    for j, sp in enumerate(specs):
        a, n = int(offs[j]), int(sizes[j])
        if sp.kind == "normal":
            z = torch.randn(n, device="cuda", generator=gen) * sp.sigma + sp.mu
            arena[a:a + n] = z.round().clamp_(0, 255).to(torch.uint8)
        elif sp.kind == "spike":
            m = torch.rand(n, device="cuda", generator=gen) < 0.9
            arena[a:a + n].masked_fill_(m, sp.value)
    return arena, offs, sizes


def test_batch_full_size_4096_images(hm):
    # the full 4096-image batch (about 3.85 GB): every one of the 4096 outputs is compared with
    # the oracle over the arena read back, after the eager launch and after two graph replays
    specs = G.batch_specs(4096)
    arena, offs, sizes = batch_arena_on_device(specs, G.ROOT_SEED + 4)
    host = arena.cpu().numpy()
    exp = O.hist_many(host, offs, sizes).astype(np.int64)
    del host
    base = int(arena.data_ptr())
    rows = np.stack([base + offs, sizes], axis=1)
    out = torch.full((4096, 256), -1, dtype=torch.int32, device="cuda")
    hm.hist_batch(rows, out, mode=hm.MODE_AUTO)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.int64), exp)
    graph = hm.BatchGraph(rows, out, mode=hm.MODE_AUTO)
    for rep in range(2):
        out.fill_(-1)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().astype(np.int64), exp), rep
    graph.close()


def test_batch_errors(hm):
    out = torch.zeros((2, 256), dtype=torch.int32, device="cuda")
    with pytest.raises(hm.HistError) as e:
        hm.hist_batch([(0, 10), (0, 0)], out)
    assert e.value.status == hm.EINVAL
    with pytest.raises(hm.HistError) as e:
        hm.hist_batch([(int(out.data_ptr()), 1 << 32)], out)
    assert e.value.status == hm.EOVERFLOW


@pytest.mark.parametrize("n", [0, 5, 300_000, 5 << 20])
def test_batch_of_one(hm, n):
    # a one-buffer batch goes through the descriptor table like any other batch
    host = G.uniform_bytes(n + 3, G.rng(6, n))
    for mode in (hm.MODE_AUTO, hm.MODE_WAVEHIST):
        got = run_batch(hm, host, [3], [n], mode)
        assert np.array_equal(got[0], O.hist(host[3:3 + n]).astype(np.int64)), (n, mode)


@pytest.mark.parametrize("mode", [0, 2])
def test_batch_one_large_among_many_tiny(hm, mode):
    # equal byte shares: one 64 MiB image splits over many workgroups while the shares at
    # either side hold hundreds of tiny images each; passed as an (n, 2) array of rows
    g = np.random.default_rng(4242)
    sizes = [int(x) for x in g.integers(0, 3000, 1000)] + [64 << 20] + [int(x) for x in g.integers(0, 3000, 1000)]
    sizes[5] = sizes[1500] = 0
    offs = np.zeros(len(sizes), dtype=np.int64)
    offs[1:] = np.cumsum(sizes)[:-1]
    arena = np.concatenate([G.uniform_bytes(n, g) if k % 3 else G.constant_bytes(n, k % 256)
                            for k, n in enumerate(sizes)])
    d = dev(arena)
    rows = np.stack([int(d.data_ptr()) + offs, np.array(sizes, dtype=np.int64)], axis=1)
    out = torch.full((len(sizes), 256), -1, dtype=torch.int32, device="cuda")
    hm.hist_batch(rows, out, mode=mode)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    for k, (o, n) in enumerate(zip(offs, sizes)):
        assert np.array_equal(got[k], O.hist(arena[o:o + n]).astype(np.int64)), k
