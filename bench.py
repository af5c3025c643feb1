"""Benchmark of the adaptive-histogram hot path on one MI355X.

One step = one pass of a single stream of 66 chunks x 4 MiB (264 MiB of 8-bit pixels:
clipped Normal(128, sigma) chunks with sigma 96/32/8/2, a fully degenerate chunk and a
two-spike chunk) through the device-resident stream: per-chunk exact histograms, the
Accumulator, the moving window, the degeneracy switch and the pattern recomputation, all in
one persistent launch.  Chunk k + 1 runs with the decision made from chunk k (lag 0).
Inputs are resident in HBM before timing starts; four copies of the stream are used in turn
so no step reads bytes the 256 MB cache just saw.  Consecutive steps go to two HIP streams
in turn: the next launch fills the device while the previous one drains (the paper
pipelines its stream over several CUDA streams the same way).

Prints ONE JSON line.  Extra fields: a roofline of the dominant kernel (algorithmic bytes
per launch over the launch's share of the device: the mean interval between successive
launch completions, from HIP events recorded on the launching HIP streams), the CPU
oracle timed on the host's cores, the same stream at the tuned pipeline lag and with the
paper's 960-entry sub-histogram, a 1 MiB single image, and the 8192 x 8192 input matrix of
the paper's Table 2.
"""

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
SERVER_HIP_STREAMS = 4   # HIP streams the served bench's micro-batches are spread over
MIB = 1 << 20
N_ARENAS = 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--lag", type=int, default=0, help="pipeline lag of the headline stream (0: chunk k + 1 "
                    "runs with the decision from chunk k)")
    ap.add_argument("--theta", type=int, default=None)
    ap.add_argument("--S", type=int, default=None)
    ap.add_argument("--rmax", type=int, default=None)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (calibrates HBM byte counters)")
    ap.add_argument("--lds-probe", action="store_true",
                    help="only run each counting kernel once on the 64 MiB Table 2 inputs (for LDS counters)")
    return ap.parse_args()


def copy_probe():
    """A plain copy of known size: 256 MiB read + 256 MiB written per dispatch, 3 dispatches."""
    import torch
    n = 256 * MIB
    src = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read_per_dispatch": n, "copy_probe_bytes_written_per_dispatch": n,
                      "dispatches": 3}), flush=True)


def lds_probe():
    """One launch per (input, kernel) on the paper's 8192 x 8192 matrix (Table 2), in a fixed
    order that the printed JSON lists, for per-dispatch LDS counters (bank and address
    conflicts, LDS busy and wait cycles)."""
    import torch

    import paper_1011_0235_amd as hm
    import synthgen as G
    from oracle import oracle as O
    hm.load()
    kernels = [("uniform_r32", hm.MODE_AUTO, None), ("wavehist", hm.MODE_WAVEHIST, None),
               ("waveagg", hm.MODE_WAVEAGG, None), ("paper960", hm.MODE_AHIST, hm.pattern_init(hm.PAT_PAPER960))]
    out = torch.zeros(256, dtype=torch.int32, device="cuda")
    order, ok = [], True
    for kind in ("random", "all127", "xray"):
        host = G.table2_input(kind)
        d = torch.from_numpy(host).cuda()
        exp = O.hist(host).astype(np.int64)
        for name, mode, pat in kernels:
            hm.hist_u8(d, out, mode=mode, pattern=pat)
            torch.cuda.synchronize()
            ok = ok and bool(np.array_equal(out.cpu().numpy().astype(np.int64), exp))
            order.append("%s/%s" % (kind, name))
        del d
    print(json.dumps({"lds_probe_dispatch_order": order, "bytes_per_dispatch": 64 * MIB, "parity_exact": ok}),
          flush=True)


def profiled_traffic():
    """HBM bytes per launch from the committed counter profile, if the kernel is unchanged since."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "histmi_dev.h"):
        with open(os.path.join(ROOT, "paper_1011_0235_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    p = os.path.join(ROOT, "profiles", "hist_main_stream_66x4MiB.md")
    if not os.path.exists(p):
        return None
    text = open(p).read()
    if h.hexdigest() not in text:
        return None
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch:"):
            return int(line.split(":")[1])
    return None


def timed(torch, stream, fn, reps):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_config2(hm, O, chunks, exp, bufs, run_stream, stream):
    """The single stream as the scope's config 2 fixes it: the switch decided by the data
    (theta 45, W = 1, the paper's 960-entry sub-histogram budget with at most 8 sub-bins per
    value), at lag 0 (chunk k + 1 runs with the decision from chunk k) and lag 1.  Each lag:
    8 timed steps of the whole stream in auto, forced AHist and forced per-wavefront modes
    (two HIP streams in turn), then one traced push of the 66 chunks on one HIP stream whose
    mode and pattern traces are checked against the oracle at the same lag and whose device
    timeline gives the interval between consecutive chunk completions, the decision wait
    (lag 0: a chunk's first workgroup's start after the previous chunk's decision) and the
    counting time (start to end).  At lag 0 the chunks finish in order, so the interval is
    each chunk's own time and gives its rate; from lag 1 on, chunk k + 1 no longer waits for
    chunk k and neighbours overlap, so only the completion intervals are reported."""
    import torch
    S, rmax, theta = 960, 8, 45
    n = len(chunks)
    nbytes = int(sum(c.size for c in chunks))
    res = {"S": S, "rmax": rmax, "theta_pct": theta, "W": 1}
    for lag in (0, 1):
        row = {}
        for name, mode in (("auto", hm.MODE_AUTO), ("forced_ahist", hm.MODE_AHIST),
                           ("forced_wavehist", hm.MODE_WAVEHIST)):
            # every chunk of the 3 + 8 pushes is traced: the device timeline of the 8 timed
            # ones shows the per-chunk time and the rate of the shader's cycle counter inside
            # the finalizers (which falls with the engine clock)
            st = hm.Stream(W=1, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=11 * n)
            d0 = hm.diag()
            tms = run_stream(st, 8, 3, n_hip=2, mode=mode)
            d1 = hm.diag()
            tt = st.read_times(11 * n).astype(np.int64)[3 * n:]
            st.close()
            row[name + "_GBps"] = round(nbytes * 8 / (tms * 1e-3) / 1e9, 1)
            dt = np.diff(np.sort(tt[:, 1])) / 1e3   # between consecutive completions
            row[name + "_us_per_chunk_p50_p90_max"] = [round(float(x), 2) for x in
                                                        (np.median(dt), np.percentile(dt, 90), dt.max())]
            row[name + "_cycle_counter_MHz_p10_p50_p90"] = [int(x) for x in np.percentile(tt[:, 2], [10, 50, 90])]
            if d1.wait_timeouts != d0.wait_timeouts:
                row[name + "_wait_timeouts"] = int(d1.wait_timeouts - d0.wait_timeouts)
        st = hm.Stream(W=1, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=n)
        out = torch.zeros((n, 256), dtype=torch.int32, device="cuda")
        st.push_many(bufs, d_out=out, stream=stream)
        tt = st.read_times(n, stream=stream).astype(np.int64)
        _, modes, pats = st.read(n, stream=stream)
        st.close()
        ref = O.stream_reference(None, W=1, theta_pct=theta, S=S, rmax=rmax, lag=lag, hists=list(exp))
        ok = (bool(np.array_equal(out.cpu().numpy().astype(np.int64), exp))
              and [int(m) for m in modes] == ref["modes"]
              and [list(map(int, p)) for p in pats] == ref["patterns"])
        ends, starts = tt[:, 1], tt[:, 0]
        in_order = bool(np.all(np.diff(ends) > 0))
        per_chunk_us = np.diff(np.sort(ends)) / 1e3            # between consecutive completions
        count_us = (ends - starts) / 1e3
        row["traced_push"] = {
            "chunks_finish_in_order": in_order,
            "us_per_chunk_p10_p50_p90": [round(float(x), 2) for x in np.percentile(per_chunk_us, [10, 50, 90])],
            "cycle_counter_MHz_p10_p50_p90": [int(x) for x in np.percentile(tt[:, 2], [10, 50, 90])],
            "count_us_p50": round(float(np.median(count_us)), 2)}
        if in_order:
            row["traced_push"]["per_chunk_GBps"] = [round(c.size / (u * 1e-6) / 1e9, 1)
                                                    for c, u in zip(chunks[1:], per_chunk_us)]
        row["traced_push"].update({
            "mode_trace": "".join("A" if m == hm.MODE_AHIST else "W" for m in ref["modes"]),
            "parity_exact": ok})
        if lag == 0:
            wait_us = (starts[1:] - ends[:-1]) / 1e3
            row["traced_push"]["decision_wait_us_p10_p50_p90"] = [
                round(float(x), 2) for x in np.percentile(wait_us, [10, 50, 90])]
        res["lag%d" % lag] = row
    return res


def bench_batched(hm, G, O, torch, dev, stream):
    """The 4096-image batch (sides log-uniform 64..4096; uniform / Normal / 90 % spike images), generated
    on the device: one persistent launch, the same launch replayed from a HIP graph, and 4096 sequential
    single-image launches."""
    specs = G.batch_specs(4096)
    sizes = np.array([sp.size for sp in specs], dtype=np.int64)
    offs = np.zeros_like(sizes)
    offs[1:] = np.cumsum((sizes + 255) // 256 * 256)[:-1]
    total = int(offs[-1] + sizes[-1])
    gen = torch.Generator(device=dev)
    gen.manual_seed(G.ROOT_SEED + 4)
    arena = torch.randint(0, 256, (total,), dtype=torch.uint8, device=dev, generator=gen)
    for j, sp in enumerate(specs):
        a, n = int(offs[j]), int(sizes[j])
        if sp.kind == "normal":
            z = torch.randn(n, device=dev, generator=gen) * sp.sigma + sp.mu
            arena[a:a + n] = z.round().clamp_(0, 255).to(torch.uint8)
        elif sp.kind == "spike":
            m = torch.rand(n, device=dev, generator=gen) < 0.9
            arena[a:a + n].masked_fill_(m, sp.value)
    base = int(arena.data_ptr())
    bufs = [(base + int(o), int(n)) for o, n in zip(offs, sizes)]
    rows = np.stack([base + offs, sizes], axis=1)   # the same buffers as one (4096, 2) array
    out = torch.zeros((4096, 256), dtype=torch.int32, device=dev)
    nb = int(sizes.sum())
    # the first call also allocates the library's scratch and staging for a batch of this shape:
    # reported on its own, then twenty calls in steady state (the host plans each call while
    # the device runs the one before; only the first call's planning falls in the timed region)
    ms_first = timed(torch, stream, lambda: hm.hist_batch(rows, out, mode=hm.MODE_AUTO, stream=stream), 1)
    ms_batch = timed(torch, stream, lambda: hm.hist_batch(rows, out, mode=hm.MODE_AUTO, stream=stream), 20)
    got_eager = out.cpu().numpy().astype(np.int64)
    out.fill_(-1)
    graph = hm.BatchGraph(rows, out, mode=hm.MODE_AUTO)
    ms_graph = timed(torch, stream, lambda: graph.launch(stream=stream), 20)
    got_graph = out.cpu().numpy().astype(np.int64)
    graph.close()
    # every one of the 4096 outputs of both launches against the oracle over the arena read back
    exp = O.hist_many(arena.cpu().numpy(), offs, sizes).astype(np.int64)
    ok = bool(np.array_equal(got_eager, exp)) and bool(np.array_equal(got_graph, exp))
    outs1 = [out[j] for j in range(4096)]

    def seq():
        for j in range(4096):
            hm.hist_u8(bufs[j][0], outs1[j], mode=hm.MODE_AUTO, stream=stream, n=bufs[j][1])
    ms_seq = timed(torch, stream, seq, 1)
    del arena
    return {"images": 4096, "bytes": nb,
            "persistent_GBps": round(nb / (ms_batch * 1e-3) / 1e9, 1), "persistent_ms": round(ms_batch, 3),
            "persistent_first_call_ms": round(ms_first, 3),
            "graph_GBps": round(nb / (ms_graph * 1e-3) / 1e9, 1), "graph_ms": round(ms_graph, 3),
            "sequential_hist_u8_GBps": round(nb / (ms_seq * 1e-3) / 1e9, 1), "sequential_ms": round(ms_seq, 3),
            "speedup_vs_sequential": round(ms_seq / ms_graph, 2), "parity_exact": ok}


def bench_xray(hm, G, O, torch, dev, hip_streams, S, rmax, lag, plag, theta, frames=512):
    """The X-ray-like frame stream (512 frames of 2048 x 2048, 2 GiB): the mean of each frame's
    clipped Normal walks (step sigma 4), its sigma is U[6, 40], 1 % of its pixels are saturated.
    Generated on the device under the root seed; all frames are pushed in one launch, the
    pattern carried on the device.  The mode and pattern traces of one pass are checked
    exactly against the oracle's stream reference (per-frame histograms of the bytes read
    back); then the pass is timed, alternating two HIP streams."""
    n = 2048 * 2048
    specs = G.xray_specs(frames)
    gen = torch.Generator(device=dev)
    gen.manual_seed(G.ROOT_SEED + 3)
    arena = torch.empty(frames * n, dtype=torch.uint8, device=dev)
    k_sat = int(round(0.01 * n))
    for t, sp in enumerate(specs):
        z = torch.randn(n, device=dev, generator=gen) * sp.sigma + sp.mu
        fr = arena[t * n:(t + 1) * n]
        fr.copy_(z.round_().clamp_(0, 255).to(torch.uint8))
        fr[torch.randperm(n, device=dev, generator=gen)[:k_sat]] = 255
    torch.cuda.synchronize()
    host = arena.cpu().numpy()
    hists = [O.hist(host[t * n:(t + 1) * n]) for t in range(frames)]
    del host
    base = int(arena.data_ptr())
    bufs = [(base + t * n, n) for t in range(frames)]
    outs = [torch.zeros((frames, 256), dtype=torch.int32, device=dev) for _ in range(2)]
    exp = np.stack(hists).astype(np.int64)
    res = {"frames": frames, "bytes": frames * n}
    # (the data-dependent switches at theta 45 and 4 run at the tuned pipeline lag: at lag 0
    # every frame would wait for the decision from the frame before it)
    for name, (th, lg, mode) in {"auto": (theta, lag, hm.MODE_AUTO), "ahist": (theta, lag, hm.MODE_AHIST),
                                 "wavehist": (theta, lag, hm.MODE_WAVEHIST),
                                 "auto_lag%d" % plag: (theta, plag, hm.MODE_AUTO),
                                 "auto_theta45_lag%d" % plag: (45, plag, hm.MODE_AUTO),
                                 "auto_theta4_lag%d" % plag: (4, plag, hm.MODE_AUTO)}.items():
        ref = O.stream_reference(None, W=1, theta_pct=th, S=S, rmax=rmax, lag=lg, hists=hists, mode=mode)
        st = hm.Stream(W=1, theta_pct=th, S=S, rmax=rmax, lag=lg, trace_cap=frames)
        st.push_many(bufs, mode=mode, d_out=outs[0], stream=hip_streams[0])
        _, modes, pats = st.read(frames, stream=hip_streams[0])
        ok = (bool(np.array_equal(outs[0].cpu().numpy().astype(np.int64), exp))
              and [int(m) for m in modes] == ref["modes"]
              and [list(map(int, p)) for p in pats] == ref["patterns"])
        reps = 4
        for r in range(2):   # untimed: the launch shapes, descriptors and clocks settle
            st.push_many(bufs, mode=mode, d_out=outs[r & 1], stream=hip_streams[r & 1])
        # timed as the headline: a start event on the first launch's HIP stream, the later of
        # the two HIP streams' end events
        e0 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(hip_streams[0])
        hip_streams[1].wait_event(e0)
        for r in range(reps):
            st.push_many(bufs, mode=mode, d_out=outs[r & 1], stream=hip_streams[r & 1])
        ends = []
        for h in hip_streams:
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(h)
            ends.append(ev)
        torch.cuda.synchronize()
        ms = max(e0.elapsed_time(ev) for ev in ends) / reps
        st.close()
        n_ahist = sum(1 for m in ref["modes"] if m == hm.MODE_AHIST)
        switches = sum(1 for a, b in zip(ref["modes"], ref["modes"][1:]) if a != b)
        res[name] = {"GB/s": round(frames * n / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 3), "theta_pct": th,
                     "lag": lg, "frames_ahist": n_ahist, "mode_switches": switches, "parity_exact": ok}
    del arena
    return res


def bench_ingest(hm, G, O, torch, dev):
    """The stream fed from HOST memory (the paper's Sec. III.B setting): the 66 x 4 MiB stream in
    pinned host memory, with the paper's pattern budget (S 960, rmax 8, theta 45) and the
    pattern of chunk k+1 from chunk k (lag 0).
    Sequential (Tables 3-4): one HIP stream; per chunk the host-to-device copy, the chunk's
    launch and the copy of its histogram back to pinned host memory, then a host
    synchronisation.  HIP events around each of the three split the device time, and the
    rest of each chunk's wall time is the host's (launch calls, synchronisation, event
    records): the columns partition the sequential time.  The paper's CPU pattern
    recomputation is zero here: the device makes every decision.
    Pipelined (Figs. 3-4): hist_ingest over 1..256 HIP streams (W = 1, the Accumulator;
    moving windows W = 32 / 128 / 256), as % of the sequential time; the device timeline of
    the best pass gives the longest gap between one chunk's end and the next chunk's start."""
    chunks = G.stream_chunks(4 * MIB)
    n = 4 * MIB
    nch = len(chunks)
    host = torch.empty(nch * n, dtype=torch.uint8, pin_memory=True)
    hv = host.numpy()
    for k, c in enumerate(chunks):
        hv[k * n:(k + 1) * n] = c
    base = int(host.data_ptr())
    exp = np.stack([O.hist(c) for c in chunks]).astype(np.int64)
    nb = nch * n
    outs = torch.zeros((nch, 256), dtype=torch.int32, device=dev)
    hout = torch.zeros((nch, 256), dtype=torch.int32, pin_memory=True)
    dcopy = torch.empty(n, dtype=torch.uint8, device=dev)
    cur = torch.cuda.current_stream()
    S, rmax, theta = 960, 8, 45

    def wall(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # ---- sequential, partitioned
    def sequential_pass():
        st = hm.Stream(W=1, theta_pct=theta, S=S, rmax=rmax, lag=0, trace_cap=0)
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(nch)]
        walls = []
        torch.cuda.synchronize()
        for k in range(nch):
            t0 = time.perf_counter()
            e = ev[k]
            e[0].record(cur)
            dcopy.copy_(host[k * n:(k + 1) * n], non_blocking=True)
            e[1].record(cur)
            st.push(dcopy, d_out=outs[k], stream=cur)
            e[2].record(cur)
            hout[k].copy_(outs[k], non_blocking=True)
            e[3].record(cur)
            cur.synchronize()
            walls.append(time.perf_counter() - t0)
        st.close()
        h2d = sum(e[0].elapsed_time(e[1]) for e in ev) * 1e-3
        kern = sum(e[1].elapsed_time(e[2]) for e in ev) * 1e-3
        d2h = sum(e[2].elapsed_time(e[3]) for e in ev) * 1e-3
        total = sum(walls)
        ok = bool(np.array_equal(hout.numpy().astype(np.int64), exp))
        return total, h2d, kern, d2h, ok

    sequential_pass()   # warm
    best = min((sequential_pass() for _ in range(3)), key=lambda x: x[0])
    t_seq, h2d, kern, d2h, ok_seq = best
    host_other = t_seq - h2d - kern - d2h
    res = {"bytes": nb, "chunks": nch, "S": S, "rmax": rmax, "theta_pct": theta, "lag": 0}
    res["sequential"] = {"ms": round(t_seq * 1e3, 3), "GB/s": round(nb / t_seq / 1e9, 2), "parity_exact": ok_seq,
                         "pct_cpu_pattern": 0.0,
                         "pct_h2d": round(100 * h2d / t_seq, 1), "pct_kernel": round(100 * kern / t_seq, 1),
                         "pct_d2h": round(100 * d2h / t_seq, 1), "pct_host": round(100 * host_other / t_seq, 1)}

    # ---- pipelined through hist_ingest
    def ingest_pass(ing, W):
        reps = 4
        st = hm.Stream(W=W, theta_pct=theta, S=S, rmax=rmax, lag=0, trace_cap=reps * nch)
        times = []
        for _ in range(reps):   # the first pass warms
            def go():
                for k in range(nch):
                    ing.push(st, base + k * n, d_out=outs[k], n=n)
                ing.sync()
            times.append(wall(go))
        ok = bool(np.array_equal(outs.cpu().numpy().astype(np.int64), exp))
        tt = st.read_times(reps * nch).astype(np.int64)
        st.close()
        b = 1 + int(np.argmin(times[1:]))
        seg = tt[b * nch:(b + 1) * nch]
        gaps = (seg[1:, 0] - seg[:-1, 1]) / 1e3
        return times[b], ok, float(gaps.max()), int(np.argmax(gaps)) + 1, int(np.median(seg[:, 2]))

    fig = {}
    for W in (1, 32, 128, 256):
        row = {}
        for K in ((1, 2, 4, 8, 16, 32, 64, 128, 256) if W == 1 else (1, 16, 256)):
            ing = hm.Ingest(n_hip_streams=K, slot_bytes=n)
            t, ok, gap_us, gap_k, mhz = ingest_pass(ing, W)
            ing.close()
            row[K] = {"pct_of_sequential": round(100 * t / t_seq, 1), "GB/s": round(nb / t / 1e9, 2),
                      "parity_exact": ok, "max_gap_us": round(gap_us, 1), "max_gap_before_chunk": gap_k,
                      "cycle_counter_MHz_p50": mhz}
        fig["W%d" % W] = row
    res["pipelined"] = fig
    res["wait_timeouts"] = int(hm.diag().wait_timeouts)   # in-kernel decision waits that gave up (0 expected)
    del host, dcopy
    return res


def drifting_pools(torch, dev, n_streams, pool_bytes, piece, seed):
    """Per-stream pools of the served workload, generated on the device: consecutive 4 MiB
    pieces of a clipped Normal whose mean walks (start U[40, 215], step sigma 4) and whose
    sigma is U[6, 40] per piece, as the X-ray-like frames."""
    g = np.random.default_rng(seed)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    out = []
    for _ in range(n_streams):
        p = torch.empty(pool_bytes, dtype=torch.uint8, device=dev)
        mu = float(g.uniform(40, 215))
        for s0 in range(0, pool_bytes, piece):
            e = min(pool_bytes, s0 + piece)
            mu = float(np.clip(mu + 4.0 * g.standard_normal(), 0.0, 255.0))
            sigma = float(g.uniform(6.0, 40.0))
            z = torch.randn(e - s0, device=dev, generator=gen) * sigma + mu
            p[s0:e] = z.round_().clamp_(0, 255).to(torch.uint8)
        out.append(p)
    return out


class PoolOracle:
    """The oracle's histogram of any slice of a pool, from the oracle's histograms of the
    pool's 16 KiB blocks (prefix sums) plus its histograms of the slice's partial blocks at
    either end: counts add over concatenation, so this is exact."""
    B = 16384

    def __init__(self, O, host_pool):
        self.O = O
        self.pool = host_pool
        nb = host_pool.size // self.B
        blocks = O.hist_many(host_pool, np.arange(nb, dtype=np.uint64) * self.B,
                             np.full(nb, self.B, dtype=np.uint64)).astype(np.int64)
        self.cum = np.zeros((nb + 1, 256), dtype=np.int64)
        np.cumsum(blocks, axis=0, out=self.cum[1:])

    def hists(self, offs, sizes):
        offs = np.asarray(offs, dtype=np.int64)
        sizes = np.asarray(sizes, dtype=np.int64)
        ends = offs + sizes
        b0 = -(-offs // self.B)
        b1 = ends // self.B
        inner = b0 < b1
        out = np.zeros((offs.size, 256), dtype=np.int64)
        out[inner] = self.cum[b1[inner]] - self.cum[b0[inner]]
        # partial blocks: [off, b0 B) and [b1 B, end) when the slice spans a block boundary,
        # else the whole slice
        h_off = np.where(inner, offs, offs)
        h_len = np.where(inner, b0 * self.B - offs, sizes)
        t_off = np.where(inner, b1 * self.B, 0)
        t_len = np.where(inner, ends - b1 * self.B, 0)
        out += self.O.hist_many(self.pool, h_off.astype(np.uint64), h_len.astype(np.uint64)).astype(np.int64)
        out += self.O.hist_many(self.pool, t_off.astype(np.uint64), t_len.astype(np.uint64)).astype(np.int64)
        return out


def bench_served(hm, G, O, torch, dev, stream, theta, S, rmax, rates=(1000, 10000, 50000), duration=2.0):
    """Open-loop Poisson arrivals (sizes log-uniform 4 KiB..64 MiB, 64 stream ids, slices of
    per-stream drifting pools) into the continuous-batching server with the tuned switch;
    latency from scheduled arrival to host-observed completion, beside the plain kernel taking
    the same arrivals one synchronous hist_u8 call at a time.  Then every request of the
    largest set submitted at once (offered load unbounded): the server's capacity.  Every
    request's histogram and every stream id's running histogram are checked against the
    oracle."""
    n_streams, pool = 64, 64 * MIB
    pools = drifting_pools(torch, dev, n_streams, pool, 4 * MIB, G.ROOT_SEED + 5)
    oracles = [PoolOracle(O, p.cpu().numpy()) for p in pools]
    out = {"switch": {"theta_pct": theta, "S": S, "rmax": rmax}}
    runs = [(rate, True) for rate in rates] + [(rates[-1], False)]
    for rate, paced in runs:
        reqs = G.serve_requests(float(rate), duration, n_streams=n_streams, pool_bytes=pool, item=rate)
        outs = torch.zeros((len(reqs), 256), dtype=torch.int32, device=dev)
        ptrs = [int(pools[r.stream_id].data_ptr()) + r.offset for r in reqs]
        optr = int(outs.data_ptr())
        sv = hm.Server(hbm_budget_bytes=1 << 30, max_slots=256, n_stream_ids=n_streams, n_hip_streams=SERVER_HIP_STREAMS,
                       max_batch=64, mode=hm.MODE_AUTO, theta_pct=theta, S=S, rmax=rmax)
        subs = []      # (request index, ticket, scheduled arrival ns) of every accepted submission
        refused = 0
        t0 = time.perf_counter_ns()
        for i, r in enumerate(reqs):
            due = t0 + int(r.t_arrival * 1e9) if paced else t0
            if paced:
                while time.perf_counter_ns() < due:
                    pass
            st, tk = sv.try_submit(r.stream_id, ptrs[i], d_out=optr + 1024 * i, n=r.size)
            if st == hm.OK:
                subs.append((i, tk, due))
            else:
                refused += 1
        t_submitted = time.perf_counter_ns()
        sv.drain()
        res = [(i, sv.poll(tk), due) for i, tk, due in subs]
        stats = sv.stats()
        # steady_clock in the library and perf_counter_ns here share CLOCK_MONOTONIC
        lat = np.array([(r_.t_done_ns - due) / 1e3 for _, r_, due in res])
        span = (max(r_.t_done_ns for _, r_, _ in res) - t0) / 1e9
        done_idx = [i for i, r_, _ in res if r_.status == hm.OK]
        nbytes = sum(reqs[i].size for i in done_idx)
        got = outs.cpu().numpy().astype(np.int64)
        exp = np.zeros_like(got)
        sids = np.array([r.stream_id for r in reqs], dtype=np.int64)
        roffs = np.array([r.offset for r in reqs], dtype=np.int64)
        rsizes = np.array([r.size for r in reqs], dtype=np.int64)
        done = np.zeros(len(reqs), dtype=bool)
        done[done_idx] = True
        ok = len(done_idx) == len(reqs)
        for sid in range(n_streams):
            idx = np.nonzero(sids == sid)[0]
            if idx.size:
                exp[idx] = oracles[sid].hists(roffs[idx], rsizes[idx])
            want = exp[idx[done[idx]]].sum(axis=0)
            ok = ok and bool(np.array_equal(sv.stream_acc(sid).astype(np.int64), want))
        ok = ok and bool(np.array_equal(got, exp))
        sv.close()
        row = {"requests": len(reqs), "refused": refused, "bytes": nbytes,
               "served_GBps": round(nbytes / span / 1e9, 2),
               "p50_us": round(float(np.percentile(lat, 50)), 1), "p99_us": round(float(np.percentile(lat, 99)), 1),
               "batches": int(stats.batches), "max_concurrent_batches": int(stats.max_concurrent_batches),
               "scheduler_max_launch_us": round(stats.max_launch_ns / 1e3, 1),
               "scheduler_max_query_us": round(stats.max_query_ns / 1e3, 1),
               "parity_exact": ok}
        if paced:
            row["offered_GBps"] = round(sum(r.size for r in reqs) / duration / 1e9, 2)
            # the plain kernel: one single-image launch per request, in arrival order, back to back
            ms_fifo = timed(torch, stream, lambda: [hm.hist_u8(ptrs[i], outs[i], stream=stream, n=reqs[i].size)
                                                    for i in range(len(reqs))], 1)
            row["fifo_hist_u8_GBps"] = round(sum(r.size for r in reqs) / (ms_fifo * 1e-3) / 1e9, 1)
            # the plain kernel as a server: one thread takes the same arrivals in order, calls
            # hist_u8 for each at its arrival (or at once when behind) and synchronizes; latency
            # from scheduled arrival to the synchronize's return, queueing included
            lat_plain = np.empty(len(reqs))
            t0 = time.perf_counter_ns()
            for i, r in enumerate(reqs):
                due = t0 + int(r.t_arrival * 1e9)
                while time.perf_counter_ns() < due:
                    pass
                hm.hist_u8(ptrs[i], outs[i], stream=stream, n=r.size)
                stream.synchronize()
                lat_plain[i] = (time.perf_counter_ns() - due) / 1e3
            row["plain_sync_p50_us"] = round(float(np.percentile(lat_plain, 50)), 1)
            row["plain_sync_p99_us"] = round(float(np.percentile(lat_plain, 99)), 1)
            row["plain_parity_exact"] = bool(np.array_equal(outs.cpu().numpy().astype(np.int64), exp))
            out["%d_per_s" % rate] = row
        else:
            row["offered"] = "all %d requests of the %d/s set at once" % (len(reqs), rate)
            row["host_submit_per_s"] = round(len(reqs) / ((t_submitted - t0) / 1e9), 0)
            out["capacity_all_at_once"] = row
        del outs
    del pools
    return out


def tuned_defaults():
    """Stream settings written by the autotuner (tuning.json beside the library), else built-ins."""
    d = {"lag": 31, "theta_pct": 0, "S": 8192, "rmax": 32}
    p = os.path.join(ROOT, "paper_1011_0235_amd", "tuning.json")
    if os.path.exists(p):
        with open(p) as f:
            d.update(json.load(f).get("stream", {}))
    return d


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.lds_probe:
        lds_probe()
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(sharded, each GPU would take whole streams, or images of a batch)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1011_0235_amd as hm
    import synthgen as G

    hm.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # Python's cyclic collector stays off while the bench runs: with torch loaded one full pass
    # takes about 33 ms and would land at random inside a timed region (a 40-push region of the
    # stream lasts under 2 ms).  The bench makes no reference cycles to speak of; reference
    # counting still frees everything else.
    gc.collect()
    gc.freeze()
    gc.disable()
    info = hm.device_info()
    tune = tuned_defaults()
    lag = args.lag
    plag = tune["lag"]   # the tuned pipeline lag, for the pipelined variants in the extras
    theta = tune["theta_pct"] if args.theta is None else args.theta
    S = tune["S"] if args.S is None else args.S
    rmax = tune["rmax"] if args.rmax is None else args.rmax

    # ---- inputs: the single stream, four copies resident in HBM (1.03 GiB), used in turn so
    # that no step reads bytes read in the last 792 MiB (the device cache is 256 MB)
    chunks = G.stream_chunks(4 * MIB)
    host = np.concatenate(chunks)
    nbytes = host.size
    arenas = [torch.from_numpy(host).to(dev)]
    arenas += [arenas[0].clone() for _ in range(N_ARENAS - 1)]
    nchunk = len(chunks)
    bufs = [[(int(a.data_ptr()) + k * 4 * MIB, 4 * MIB) for k in range(nchunk)] for a in arenas]
    outs = [torch.zeros((nchunk, 256), dtype=torch.int32, device=dev) for _ in range(2)]
    stream = torch.cuda.current_stream()
    # Consecutive pushes of the stream go to two HIP streams in turn, so that one launch's tail
    # overlaps the next launch's start (the library lets two launches of one stream run at
    # once; each chunk waits on the device for the decision it runs with).
    hip_streams = [torch.cuda.Stream(), torch.cuda.Stream()]

    def run_stream(st, steps, warmup, n_hip=2, mode=None):
        """Time `steps` pushes of the whole stream after `warmup` untimed ones, alternating
        n_hip HIP streams.  The region starts with an event on the first timed launch's HIP
        stream (the other one waits for it before its first timed launch) and ends with the
        later of the two streams' end events: nothing but kernels between the launches."""
        mode = hm.MODE_AUTO if mode is None else mode
        for i in range(warmup):
            st.push_many(bufs[i % N_ARENAS], mode=mode, d_out=outs[i & 1], stream=hip_streams[(i & 1) % n_hip])
        torch.cuda.synchronize()
        used = [hip_streams[((warmup + i) & 1) % n_hip] for i in range(min(steps, n_hip))]
        t_start = torch.cuda.Event(enable_timing=True)
        t_start.record(used[0])
        for h in used[1:]:
            h.wait_event(t_start)
        for i in range(steps):
            j = warmup + i   # arenas, outputs and HIP streams rotate as in the warm-up
            st.push_many(bufs[j % N_ARENAS], mode=mode, d_out=outs[j & 1], stream=hip_streams[(j & 1) % n_hip])
        t_end = []
        for h in used:
            e = torch.cuda.Event(enable_timing=True)
            e.record(h)
            t_end.append(e)
        torch.cuda.synchronize()
        return max(t_start.elapsed_time(e) for e in t_end)

    # ---- headline (no event between the timed launches: each would add a packet, and a few
    # microseconds, between kernels)
    st = hm.Stream(W=1, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_ms = run_stream(st, args.steps, args.warmup)
    wall = time.perf_counter() - t0
    ms_per_step = total_ms / args.steps
    value = nbytes * args.steps / (total_ms * 1e-3) / 1e9

    # parity of the last step's outputs against the oracle (exact)
    from oracle import oracle as O
    exp = np.stack([O.hist(c) for c in chunks]).astype(np.int64)
    parity = all(bool(np.array_equal(o.cpu().numpy().astype(np.int64), exp)) for o in outs)
    snap, _, _ = st.read(0, stream=stream)
    acc_ok = bool(np.array_equal(np.array(snap.acc, dtype=np.uint64),
                                 exp.sum(axis=0).astype(np.uint64) * (args.warmup + args.steps)))
    st.close()

    # roofline of the dominant kernel: one persistent launch per step, back to back over the
    # timed region (HIP events on the current stream, which both launching HIP streams join),
    # so a launch's average time is the timed region over the launches.  Consecutive launches
    # overlap on two HIP streams: a kernel's own start-to-end span is longer than this.
    avg_launch_ms = ms_per_step
    alg_bytes = nbytes + nchunk * 1024 + nchunk * 4096   # input + u32 outputs + u64 Accumulator read/write
    achieved = alg_bytes / (avg_launch_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(),
                "kernel": "histmi::hist_main<4>", "avg_launch_ms": round(avg_launch_ms, 5),
                "avg_launch": "timed region / launches (launches on two HIP streams in turn overlap)",
                "alg_bytes_per_launch": alg_bytes}
    # the measured read roofline: a plain streaming read of 2 x 1 GiB (used in turn), best over
    # grid sizes (streaming reads on this GPU are sensitive to the grid)
    probe = [torch.randint(0, 256, (1 << 30,), dtype=torch.uint8, device=dev) for _ in range(2)]
    psum = torch.zeros(1, dtype=torch.int64, device=dev)
    k = [0]
    read_sweep = {}
    for wg in (256, 512, 768, 1024, 2048):
        def probe_once():
            hm.read_probe(probe[k[0] & 1], psum, workgroups=wg, stream=stream)
            k[0] += 1
        read_sweep[wg] = round((1 << 30) / (timed(torch, stream, probe_once, 10) * 1e-3) / 1e9, 1)
    read_roof = max(read_sweep.values())
    del probe

    res = {
        "metric": "input GB/s and % of HBM peak (bit-exact); batched/served GB/s + p50/p99 latency",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "single stream, 66 chunks x 4 MiB (264 MiB u8): clipped Normal(128, sigma) with sigma "
                               "96/32/8/2, one all-127 chunk, one two-spike chunk; the device decides the kernel "
                               "and pattern for chunk k+1 from chunk k's histogram (lag 0), per-chunk u32 "
                               "histograms + u64 Accumulator on device.  Tuned switch: theta %d, S %d >= 256 x "
                               "rmax %d, so rule P always gives the uniform %d-sub-bin table and the test fires "
                               "for every non-empty chunk: every decision is that AHist table, known to the host "
                               "from the chunk sizes (no chunk waits); the data-dependent switch is the "
                               "config2_theta45_W1 extra" % (theta, S, rmax, rmax),
                   "chunk_bytes": 4 * MIB, "chunks": nchunk, "mode": "auto", "W": 1, "theta_pct": theta,
                   "S": S, "rmax": rmax, "lag": lag},
        "pct_of_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
        "read_roofline_GBps": round(read_roof, 1),
        "read_probe_GBps_by_workgroups": read_sweep,
        "pct_of_read_roofline": round(100.0 * value / read_roof, 2),
        "parity_exact": parity and acc_ok,
        "roofline": roofline,
        "device": {"arch": info.arch.decode(), "cus": info.cu_count, "clock_khz": info.clock_khz},
        "wall_s_timed": round(wall, 3),
    }

    # ---- CPU baseline: the oracle's plain counting loop on the host's cores
    if not args.no_cpu:
        # the host cores this process may use, at most the 16 that a one-GPU machine gives it
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        secs, reps = 0.0, 0
        while secs < max(1.0, 10.0 / threads) and reps < 200:
            t, h = O.hist_timed(host, threads)
            secs += t
            reps += 1
        assert np.array_equal(h.astype(np.int64), exp.sum(axis=0))
        # one thread too: the median of five passes
        one = sorted(O.hist_timed(host, 1)[0] for _ in range(5))[2]
        res["cpu_baseline"] = {"value": round(nbytes * reps / secs / 1e9, 3), "unit": "GB/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "the same 264 MiB stream bytes in host RAM, %d passes of the plain C "
                                         "counting loop split over %d threads (%.1f s wall; a one-GPU box gives "
                                         "a process 16 host cores)" % (reps, threads, secs),
                               "single_thread_GBps": round(nbytes / one / 1e9, 3)}

    if not args.no_extras:
        extras = {}
        extras["config2_theta45_W1"] = bench_config2(hm, O, chunks, exp, bufs[0], run_stream, stream)
        # the same stream, sequential semantics (pattern for chunk k+1 from chunk k) and paper sizes
        # (the switch exercised: theta 45 sends peaked chunks to AHist and wide ones to the
        # per-wavefront kernel; one HIP stream: no overlap between consecutive launches)
        # (moving windows of W chunks: the chunks are sequenced in order on the device; with
        # change detection on, the window is also compared with the Accumulator after every chunk)
        # (the collision criterion: entries with a kappa below use it instead of theta)
        for name, (w_, l, th, s_, r_, nh, al, *crit) in {
                "stream_lag%d_auto" % plag: (1, plag, theta, S, rmax, 2, 0),
                "stream_theta45_lag0": (1, 0, 45, S, rmax, 2, 0),
                "stream_theta45_lag%d" % plag: (1, plag, 45, S, rmax, 2, 0),
                "stream_paper960_theta45_lag0": (1, 0, 45, 960, 8, 2, 0),
                "stream_paper960_theta45_lag%d" % plag: (1, plag, 45, 960, 8, 2, 0),
                "stream_lag%d_one_hip_stream" % lag: (1, lag, theta, S, rmax, 1, 0),
                "stream_window_W32_lag%d" % plag: (32, plag, theta, S, rmax, 2, 0),
                "stream_window_W256_lag%d" % plag: (256, plag, theta, S, rmax, 2, 0),
                # a lag of one push less one chunk: every decision comes from an earlier push
                "stream_window_W32_lag65": (32, 65, theta, S, rmax, 2, 0),
                "stream_window_W32_theta45_paper960_lag%d" % plag: (32, plag, 45, 960, 8, 2, 0),
                "stream_window_W32_alarm4_lag%d" % plag: (32, plag, theta, S, rmax, 2, 4),
                "stream_alarm4_W1_lag%d" % plag: (1, plag, theta, S, rmax, 2, 4),
                "stream_collision10_W1_lag%d" % plag: (1, plag, 100, S, rmax, 2, 0, hm.CRIT_COLLISION, 10),
                "stream_collision3_W32_lag%d" % plag: (32, plag, 100, S, rmax, 2, 0, hm.CRIT_COLLISION, 3),
                "stream_collision3_W32_paper960_lag%d" % plag: (32, plag, 100, 960, 8, 2, 0, hm.CRIT_COLLISION, 3)
                }.items():
            cr, kp = (crit[0], crit[1]) if crit else (hm.CRIT_MAXBIN, 0)
            st = hm.Stream(W=w_, theta_pct=th, S=s_, rmax=r_, lag=l, trace_cap=0, alarm_pct=al, criterion=cr,
                           kappa_pct=kp)
            d0 = hm.diag()
            ksteps = 40   # as the headline: the first launch's start weighs 1/40 of the region
            tms = run_stream(st, ksteps, 4, n_hip=nh)
            d1 = hm.diag()
            row = {"GB/s": round(nbytes * ksteps / (tms * 1e-3) / 1e9, 1), "ms_per_step": round(tms / ksteps, 4)}
            # with the uniform switch (a threshold of 0, a budget of rmax sub-bins for every
            # value) each decision is a function of the chunk sizes, which the host hands to
            # the chunks (nothing waits).  A window stream then does not walk its window in the
            # counting launch: without change detection it is summed from the ring when read,
            # with it a one-workgroup launch after each push walks the chunks in order.
            # Otherwise chunks wait for the device's decisions.
            uniform = 256 * r_ <= s_ and ((cr == hm.CRIT_MAXBIN and th == 0) or (cr == hm.CRIT_COLLISION and kp == 0)
                                          or (cr == hm.CRIT_BOTH and (th == 0 or kp == 0)))
            row["decisions"] = "device" if not uniform else (
                "host (uniform switch), walked after each push" if al else
                "host (uniform switch), window summed on read" if w_ > 1 else "host (uniform switch)")
            # bounded waits that ran out (a decision or a merge): none is expected
            if d1.wait_timeouts != d0.wait_timeouts or d1.merge_timeouts != d0.merge_timeouts:
                row["wait_timeouts"] = int(d1.wait_timeouts - d0.wait_timeouts)
                row["merge_timeouts"] = int(d1.merge_timeouts - d0.merge_timeouts)
            if al:
                snap, _, _ = st.read(0)
                row["chunks"] = int(snap.chunks)
                row["alarms"] = int(snap.alarms)
            st.close()
            extras[name] = row
        # one 1 MiB image: latency of one call, back to back
        x = torch.from_numpy(G.image_1mib()).to(dev)
        o1 = torch.zeros(256, dtype=torch.int32, device=dev)
        for mode, nm in ((hm.MODE_AUTO, "auto"), (hm.MODE_WAVEHIST, "wavehist"), (hm.MODE_AHIST, "ahist_identity")):
            for _ in range(5):
                hm.hist_u8(x, o1, mode=mode, stream=stream)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(100):
                hm.hist_u8(x, o1, mode=mode, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            extras["image_1mib_us_%s" % nm] = round(e0.elapsed_time(e1) * 10.0, 2)
        # the paper's Table 2 inputs at 8192 x 8192 (64 MiB), each kernel
        t2 = {}
        pats = {"auto": (hm.MODE_AUTO, None), "wavehist": (hm.MODE_WAVEHIST, None),
                "ahist_paper960": (hm.MODE_AHIST, hm.pattern_init(hm.PAT_PAPER960))}
        for kind in G.TABLE2_KINDS:
            xs = torch.from_numpy(G.table2_input(kind)).to(dev)
            row = {}
            for nm, (mode, pat) in pats.items():
                for _ in range(3):
                    hm.hist_u8(xs, o1, mode=mode, pattern=pat, stream=stream)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                # 100 calls back to back: the host's first launch after the start event is
                # spread over all of them
                e0.record(stream)
                for _ in range(100):
                    hm.hist_u8(xs, o1, mode=mode, pattern=pat, stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                row[nm] = round(xs.numel() * 100 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
            t2[kind] = row
            del xs
        extras["table2_64mib_GBps"] = t2
        extras["xray_frames_512x4MiB"] = bench_xray(hm, G, O, torch, dev, hip_streams, S, rmax, lag, plag, theta)
        extras["host_ingest_stream"] = bench_ingest(hm, G, O, torch, dev)
        extras["batched_4096_images"] = bench_batched(hm, G, O, torch, dev, stream)
        extras["served_poisson"] = bench_served(hm, G, O, torch, dev, stream, theta, S, rmax)
        res["extras"] = extras

    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
