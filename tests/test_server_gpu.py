"""GPU tests of the continuous-batching server: every request's histogram equals the oracle
and equals the same request run alone (tolerance 0: counts are integers); each stream id's
running uint64 histogram equals the oracle sum of its requests; admission never exceeds the
HBM budget or the slot limit; micro-batches overlap; destroy cancels queued requests."""

import threading

import numpy as np
import pytest

from oracle import oracle as O
import synthgen as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def pools(n_streams, pool_bytes):
    return [G.serve_pool(s, pool_bytes, piece=1 << 18) for s in range(n_streams)]


def requests(n, n_streams, pool_bytes, seed, size_hi=None):
    g = np.random.default_rng(seed)
    hi = size_hi or pool_bytes
    out = []
    for _ in range(n):
        size = int(np.floor(np.exp(g.uniform(np.log(1), np.log(hi)))))
        if g.random() < 0.05:
            size = 0
        sid = int(g.integers(0, n_streams))
        off = int(g.integers(0, pool_bytes - size + 1))
        out.append((sid, off, size))
    return out


def test_alone_equals_mix_equals_oracle(hm):
    n_streams, pool_bytes = 8, 4 << 20
    hp = pools(n_streams, pool_bytes)
    dp = [torch.from_numpy(p).cuda() for p in hp]
    reqs = requests(400, n_streams, pool_bytes, 1)
    # alone: one hist_u8 per request
    alone = torch.zeros((len(reqs), 256), dtype=torch.int32, device="cuda")
    for i, (sid, off, n) in enumerate(reqs):
        hm.hist_u8(int(dp[sid].data_ptr()) + off, alone[i], n=n)
    torch.cuda.synchronize()
    # mixed: all through the server at once, submitted from two threads
    sv = hm.Server(hbm_budget_bytes=8 << 20, max_slots=64, n_stream_ids=n_streams, n_hip_streams=3, max_batch=16,
                   S=960, rmax=8)
    mix = torch.full((len(reqs), 256), -1, dtype=torch.int32, device="cuda")
    tickets = [0] * len(reqs)

    def submit(part):
        for i in part:
            sid, off, n = reqs[i]
            tickets[i] = sv.submit(sid, int(dp[sid].data_ptr()) + off, d_out=mix[i], n=n)

    th = [threading.Thread(target=submit, args=(range(k, len(reqs), 2),)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    sv.drain()
    for i, tk in enumerate(tickets):
        r = sv.poll(tk)
        assert r.status == hm.OK and r.bytes == reqs[i][2]
        assert r.t_submit_ns <= r.t_admit_ns <= r.t_done_ns
    a = alone.cpu().numpy().astype(np.int64)
    m = mix.cpu().numpy().astype(np.int64)
    assert np.array_equal(a, m)
    for i, (sid, off, n) in enumerate(reqs[:60]):
        assert np.array_equal(m[i], O.hist(hp[sid][off:off + n]).astype(np.int64)), i
    for s in range(n_streams):
        exp = np.zeros(256, dtype=np.uint64)
        for (sid, off, n) in reqs:
            if sid == s:
                exp += O.hist(hp[s][off:off + n])
        assert np.array_equal(sv.stream_acc(s), exp), s
    st = sv.stats()
    assert st.completed == len(reqs) and st.canceled == 0
    assert st.max_inflight_bytes <= 8 << 20 and st.max_inflight_requests <= 64
    sv.close()


def test_budget_and_slots_bound_admission(hm):
    pool = torch.randint(0, 256, (8 << 20,), dtype=torch.uint8, device="cuda")
    sv = hm.Server(hbm_budget_bytes=3 << 20, max_slots=5, n_stream_ids=2, n_hip_streams=2, max_batch=4)
    outs = torch.zeros((200, 256), dtype=torch.int32, device="cuda")
    tks = []
    g = np.random.default_rng(2)
    for i in range(200):
        n = int(g.integers(1, 1 << 20))
        tks.append(sv.submit(i % 2, int(pool.data_ptr()), d_out=outs[i], n=n))
    # a request above the budget can never be admitted
    st, _ = sv.try_submit(0, int(pool.data_ptr()), n=(3 << 20) + 1)
    assert st == hm.EINVAL
    sv.drain()
    s = sv.stats()
    assert s.completed == 200
    assert s.max_inflight_bytes <= 3 << 20 and s.max_inflight_requests <= 5
    assert s.max_concurrent_batches >= 1
    # the scheduler's longest launch and completion query were timed (and are plausible)
    assert 0 < s.max_launch_ns < 10 ** 9 and 0 < s.max_query_ns < 10 ** 9
    host = pool.cpu().numpy()
    o = outs.cpu().numpy().astype(np.int64)
    for i in (0, 1, 57, 199):
        n = int(sv.poll(tks[i]).bytes)
        assert np.array_equal(o[i], O.hist(host[:n]).astype(np.int64))
    sv.close()


def test_scheduler_wakes_after_blocking(hm):
    # with a 1 us idle spin the scheduler blocks between these requests, so each one is
    # admitted by a wake-up from submit; results and running histograms stay exact
    import time
    pool = torch.randint(0, 256, (4 << 20,), dtype=torch.uint8, device="cuda")
    host = pool.cpu().numpy()
    sv = hm.Server(hbm_budget_bytes=64 << 20, max_slots=8, n_stream_ids=2, n_hip_streams=2, max_batch=4,
                   idle_spin_us=1)
    outs = torch.zeros((12, 256), dtype=torch.int32, device="cuda")
    sizes = [1, 4096, 1 << 20, 3 << 20, 17, 65536, 4 << 20, 12345, 0, 2 << 20, 999, 1 << 16]
    want_acc = [np.zeros(256, dtype=np.int64) for _ in range(2)]
    for i, n in enumerate(sizes):
        time.sleep(0.003)           # well beyond the spin: the scheduler is blocked here
        t = sv.submit(i % 2, pool, d_out=outs[i], n=n)
        r = sv.wait(t)
        assert r.status == hm.OK and r.bytes == n
        want_acc[i % 2] += O.hist(host[:n]).astype(np.int64)
    torch.cuda.synchronize()
    got = outs.cpu().numpy().astype(np.int64)
    for i, n in enumerate(sizes):
        assert np.array_equal(got[i], O.hist(host[:n]).astype(np.int64)), n
    for sid in range(2):
        assert np.array_equal(sv.stream_acc(sid).astype(np.int64), want_acc[sid])
    sv.close()
    # the spin's upper bound is enforced
    with pytest.raises(hm.HistError):
        hm.Server(n_stream_ids=1, idle_spin_us=10 ** 7 + 1)


def test_wait_poll_and_cancel(hm):
    pool = torch.randint(0, 256, (64 << 20,), dtype=torch.uint8, device="cuda")
    sv = hm.Server(hbm_budget_bytes=64 << 20, max_slots=1, n_stream_ids=1, n_hip_streams=1, max_batch=1)
    tks = [sv.submit(0, pool, n=64 << 20) for _ in range(50)]
    r = sv.wait(tks[0])
    assert r.status == hm.OK
    # a ticket whose final state was reported is retired
    with pytest.raises(hm.HistError) as e:
        sv.poll(tks[0])
    assert e.value.status == hm.EINVAL
    r = sv.poll(tks[-1])                 # still queued: reported, not retired
    assert r.status == hm.EBUSY
    assert sv.poll(tks[-1]).status == hm.EBUSY
    # bad ids and tickets
    st, _ = sv.try_submit(5, pool, n=16)
    assert st == hm.EINVAL
    with pytest.raises(hm.HistError):
        sv.poll(10 ** 9)
    sv.close()                      # cancels what is still queued, waits for the running batch
    # a fresh server still works
    sv2 = hm.Server(n_stream_ids=1)
    out = torch.zeros(256, dtype=torch.int32, device="cuda")
    t = sv2.submit(0, pool, d_out=out, n=1 << 20)
    assert sv2.wait(t).status == hm.OK
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.int64), O.hist(pool[:1 << 20].cpu().numpy()).astype(np.int64))
    sv2.close()


def test_server_decisions_stay_exact_under_degenerate_streams(hm):
    # streams alternate degenerate and wide requests so decisions flip between kernels while
    # requests of the same stream are in flight together
    n = 1 << 18
    bufs = [torch.full((n,), 7, dtype=torch.uint8, device="cuda"),
            torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda")]
    hosts = [b.cpu().numpy() for b in bufs]
    sv = hm.Server(hbm_budget_bytes=64 << 20, max_slots=128, n_stream_ids=4, n_hip_streams=4, max_batch=8,
                   theta_pct=45, S=960, rmax=8)
    outs = torch.zeros((300, 256), dtype=torch.int32, device="cuda")
    kinds = []
    for i in range(300):
        k = (i // 3) % 2
        kinds.append(k)
        sv.submit(i % 4, bufs[k], d_out=outs[i])
    sv.drain()
    o = outs.cpu().numpy().astype(np.int64)
    ref = [O.hist(h).astype(np.int64) for h in hosts]
    for i in range(300):
        assert np.array_equal(o[i], ref[kinds[i]]), i
    assert hm.diag().wait_timeouts == 0
    sv.close()


def drifting_pools_on_device(n_streams, pool_bytes, piece, seed):
    """Per-stream pools of config-5 shape, generated on the device: consecutive pieces of a
    clipped Normal whose mean walks (step sigma 4, start U[40, 215]) and whose sigma is
    U[6, 40] per piece."""
    g = np.random.default_rng(seed)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    out = []
    for _ in range(n_streams):
        p = torch.empty(pool_bytes, dtype=torch.uint8, device="cuda")
        mu = float(g.uniform(40, 215))
        for s in range(0, pool_bytes, piece):
            e = min(pool_bytes, s + piece)
            mu = float(np.clip(mu + 4.0 * g.standard_normal(), 0.0, 255.0))
            sigma = float(g.uniform(6.0, 40.0))
            z = torch.randn(e - s, device="cuda", generator=gen) * sigma + mu
            p[s:e] = z.round_().clamp_(0, 255).to(torch.uint8)
        out.append(p)
    return out


@pytest.fixture(scope="module")
def config5_workload(hm):
    """Device pools, requests and the oracle's histogram of every request (made once)."""
    n_streams, pool = 64, 64 << 20
    dp = drifting_pools_on_device(n_streams, pool, 4 << 20, G.ROOT_SEED + 55)
    reqs = G.serve_requests(600.0, 0.5, n_streams=n_streams, pool_bytes=pool, item=77)
    exp = np.zeros((len(reqs), 256), dtype=np.int64)
    for sid in range(n_streams):
        idx = [i for i, r in enumerate(reqs) if r.stream_id == sid]
        if idx:
            host = dp[sid].cpu().numpy()
            exp[idx] = O.hist_many(host, [reqs[i].offset for i in idx], [reqs[i].size for i in idx]).astype(np.int64)
    yield n_streams, dp, reqs, exp
    del dp


@pytest.mark.parametrize("theta,S,rmax,max_batch", [(0, 8192, 32, 64), (45, 960, 8, 64), (45, 960, 8, 1)])
def test_config5_sizes_every_request_exact(hm, config5_workload, theta, S, rmax, max_batch):
    """Requests of the served workload's shape: sizes log-uniform in [4 KiB, 64 MiB], 64 stream
    ids, each a slice of its stream's drifting pool of 64 MiB; the first half arrives as a
    Poisson stream (mostly one request per micro-batch), the rest at once.  Every request's
    histogram and every stream id's running histogram equal the oracle's."""
    n_streams, dp, reqs, exp = config5_workload
    assert len(reqs) > 200
    sv = hm.Server(hbm_budget_bytes=1 << 30, max_slots=256, n_stream_ids=n_streams, n_hip_streams=4,
                   max_batch=max_batch, mode=hm.MODE_AUTO, theta_pct=theta, S=S, rmax=rmax)
    out = torch.full((len(reqs), 256), -1, dtype=torch.int32, device="cuda")
    tickets = []
    import time
    t0 = time.perf_counter()
    half = len(reqs) // 2
    for i, r in enumerate(reqs):
        if i < half:
            while time.perf_counter() - t0 < r.t_arrival:
                pass
        tickets.append(sv.submit(r.stream_id, int(dp[r.stream_id].data_ptr()) + r.offset, d_out=out[i], n=r.size))
    sv.drain()
    for i, tk in enumerate(tickets):
        res = sv.poll(tk)
        assert res.status == hm.OK and res.bytes == reqs[i].size, i
    got = out.cpu().numpy().astype(np.int64)
    bad = [i for i in range(len(reqs)) if not np.array_equal(got[i], exp[i])]
    assert not bad, bad[:10]
    for sid in range(n_streams):
        want = exp[[i for i, r in enumerate(reqs) if r.stream_id == sid]].sum(axis=0)
        assert np.array_equal(sv.stream_acc(sid).astype(np.int64), want), sid
    st = sv.stats()
    assert st.completed == len(reqs) and st.canceled == 0
    sv.close()
