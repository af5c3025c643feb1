"""Autotuner: picks launch shapes, the stream's lag and sub-histogram budget, and the
degeneracy threshold for this GPU, and writes them to a tuning.json that the binding applies
when it loads the library (and that bench.py reads for the stream settings).

Sweeps (all on seeded synthetic inputs resident in HBM):
  * workgroups per CU for each kernel family, on a 1 GiB uniform buffer (two copies used in
    turn so the 256 MB cache does not serve repeats);
  * the batch tile size, on the 4096-image batch shape;
  * the stream pipeline: lag and (S, rmax), on the 66 x 4 MiB single stream;
  * Figure 5 of the paper re-measured here: throughput of each kernel on a mixture of a
    degenerate part (fraction d, one value) and a uniform part, for d = 0..100 %.  The
    crossover -- the smallest d at which AHist with the pattern derived from that data beats
    the per-wavefront kernel -- is the tuned critical degeneracy theta (Sec. III.C).

Usage: python -m paper_1011_0235_amd.autotune --out tuning.json
"""

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MIB = 1 << 20
FAMILY = {"wavehist": 0, "uniform": 1, "lookup": 2, "waveagg": 3, "stream": 4, "stream_known": 5}


def log(*a):
    print(*a, flush=True)


def timed(torch, fn, reps, streams=()):
    """Mean ms per call of fn; `streams` are further HIP streams fn launches on (forked from
    and joined back into the current stream around the timed calls).  fn runs untimed first
    until every one of those streams has seen a launch (a HIP stream's first launch sets up
    its queue, which takes milliseconds)."""
    s = torch.cuda.current_stream()
    for _ in range(max(2, 2 * len(streams))):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for h in streams:
        h.wait_event(e0)
    for _ in range(reps):
        fn()
    for h in streams:
        ev = torch.cuda.Event()
        ev.record(h)
        s.wait_event(ev)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def rule_p_host(h, S, rmax):
    """Rule P for a host pattern argument, computed on the device by hist_pattern_update."""
    import torch

    import paper_1011_0235_amd as hm
    dh = torch.from_numpy(np.asarray(h, dtype=np.int64)).cuda()
    dp = torch.zeros(258, dtype=torch.int32, device="cuda")
    hm.pattern_update(dh, S, rmax, dp)
    w = (dp.cpu().numpy().astype(np.int64) & 0xFFFFFFFF).tolist()
    return hm.Pattern.from_words(w[:256], S, rmax)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.json"))
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()

    import torch

    import paper_1011_0235_amd as hm
    import synthgen as G

    hm.load(apply_tuning=False)
    # the cyclic collector's full passes (about 33 ms with torch loaded) would land inside timed
    # regions at random; the sweeps make no reference cycles to speak of
    gc.collect()
    gc.freeze()
    gc.disable()
    dev = torch.device("cuda:0")
    result = {"device": hm.device_info().arch.decode(), "families": {}, "sweeps": {}}

    # ---- workgroups per CU per family, 1 GiB uniform, rotating copies
    g = torch.Generator(device=dev)
    g.manual_seed(G.ROOT_SEED)
    big = torch.randint(0, 256, (2, 1 << 30), dtype=torch.uint8, device=dev, generator=g)
    out = torch.zeros(256, dtype=torch.int32, device=dev)
    fam_modes = {"wavehist": (hm.MODE_WAVEHIST, None), "uniform": (hm.MODE_AUTO, None),
                 "lookup": (hm.MODE_AHIST, hm.pattern_init(hm.PAT_PAPER960)), "waveagg": (hm.MODE_WAVEAGG, None)}
    for fam, (mode, pat) in fam_modes.items():
        best, rows = None, {}
        for bpc in (1, 2, 3, 4):
            hm.tune_set(FAMILY[fam], blocks_per_cu=bpc)
            i = [0]

            def f():
                hm.hist_u8(big[i[0] & 1], out, mode=mode, pattern=pat)
                i[0] += 1
            ms = timed(torch, f, 6)
            gbs = (1 << 30) / ms / 1e6
            rows[bpc] = round(gbs, 1)
            if best is None or gbs > rows[best]:
                best = bpc
        hm.tune_set(FAMILY[fam], blocks_per_cu=best)
        result["families"][fam] = {"blocks_per_cu": best}
        result["sweeps"]["bpc_" + fam] = rows
        log("bpc", fam, rows, "->", best)
    del big

    # ---- batch tile size (4096-image shape, uniform bytes)
    specs = G.batch_specs(1024 if args.quick else 4096)
    sizes = np.array([s.size for s in specs], dtype=np.int64)
    offs = np.zeros_like(sizes)
    offs[1:] = np.cumsum((sizes + 255) // 256 * 256)[:-1]
    arena = torch.randint(0, 256, (int(offs[-1] + sizes[-1]),), dtype=torch.uint8, device=dev, generator=g)
    bufs = [(int(arena.data_ptr()) + int(o), int(n)) for o, n in zip(offs, sizes)]
    bout = torch.zeros((len(bufs), 256), dtype=torch.int32, device=dev)
    rows, best = {}, None
    for tk in (64, 128, 256, 512, 1024):
        hm.tune_set(FAMILY["uniform"], tile_kib=tk)
        ms = timed(torch, lambda: hm.hist_batch(bufs, bout, mode=hm.MODE_AUTO), 4)
        rows[tk] = round(int(sizes.sum()) / ms / 1e6, 1)
        if best is None or rows[tk] > rows[best]:
            best = tk
    hm.tune_set(FAMILY["uniform"], tile_kib=best)
    result["families"]["uniform"]["tile_kib"] = best
    result["sweeps"]["batch_tile_kib"] = rows
    log("batch tile", rows, "->", best)
    del arena

    # ---- stream pipeline (66 x 4 MiB)
    chunks = G.stream_chunks(4 * MIB)
    # four copies used in turn, as the bench uses them: no push reads bytes that the last
    # 792 MiB of pushes read (the device cache holds 256 MB)
    a0 = torch.from_numpy(np.concatenate(chunks)).to(dev)
    arenas = [a0] + [a0.clone() for _ in range(3)]
    sbufs = [[(int(a.data_ptr()) + k * 4 * MIB, 4 * MIB) for k in range(len(chunks))] for a in arenas]
    souts = [torch.zeros((len(chunks), 256), dtype=torch.int32, device=dev) for _ in range(2)]
    hip_streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    nb = a0.numel()

    def pusher(st):
        """One push of the whole stream per call: copies, outputs and the two HIP streams in
        turn, as the bench runs them."""
        i = [0]

        def f():
            k = i[0]
            st.push_many(sbufs[k % len(sbufs)], d_out=souts[k & 1], stream=hip_streams[k & 1])
            i[0] += 1
        return f
    rows, cfgs = {}, {}
    for S, rmax, theta in ((8192, 32, 0), (16384, 64, 0), (960, 8, 45), (960, 8, 0)):
        for lag in (0, 1, 3, 7, 15, 31, 63):
            st = hm.Stream(W=1, theta_pct=theta, S=S, rmax=rmax, lag=lag, trace_cap=0)
            ms = timed(torch, pusher(st), 10, hip_streams)
            st.close()
            key = "S%d_r%d_t%d_lag%d" % (S, rmax, theta, lag)
            rows[key] = round(nb / ms / 1e6, 1)
            cfgs[key] = {"S": S, "rmax": rmax, "theta_pct": theta, "lag": lag}
            log("stream", key, rows[key])
    # the pipelined stream at a pipeline depth of 31 chunks (with decisions the host knows in
    # advance every lag runs alike, so the depth is fixed rather than picked from noise): the
    # built-in (S 8192, rmax 32, theta 0) unless another setting beats it by more than 3 %
    best = "S8192_r32_t0_lag31"
    for k in rows:
        if cfgs[k]["lag"] == 31 and rows[k] > 1.03 * rows[best]:
            best = k
    result["sweeps"]["stream"] = rows
    result["stream"] = cfgs[best]
    log("stream ->", cfgs[best])
    # launch shapes of stream pushes: workgroups per CU x tiles per workgroup (each measured
    # in three interleaved passes of 20 pushes, the median kept).  Two families: pushes whose
    # decisions the host knows (the tuned configuration at lag 0: nothing waits) and pushes
    # whose chunks wait for the device's decisions (the paper's threshold of 45 with the
    # tuned budget at the tuned lag: tiles handed out in chunk order).
    c = cfgs[best]

    def shape_sweep(family, make, bpcs, tpws):
        shape = {}
        for rep in range(3):
            for bpc in bpcs:
                for tpw in tpws:
                    hm.tune_set(FAMILY[family], blocks_per_cu=bpc, tiles_per_wg=tpw)
                    st = make()
                    ms = timed(torch, pusher(st), 20, hip_streams)
                    st.close()
                    shape.setdefault("bpc%d_tpw%d" % (bpc, tpw), []).append(nb / ms / 1e6)
        rows = {k: round(float(np.median(v)), 1) for k, v in shape.items()}
        bk = max(rows, key=lambda k: rows[k])
        bpc, tpw = int(bk[3]), int(bk.split("tpw")[1])
        hm.tune_set(FAMILY[family], blocks_per_cu=bpc, tiles_per_wg=tpw)
        result["families"][family] = {"blocks_per_cu": bpc, "tiles_per_wg": tpw}
        result["sweeps"][family + "_shape"] = rows
        log(family, "shape", rows, "->", bk)

    shape_sweep("stream_known",
                lambda: hm.Stream(W=1, theta_pct=c["theta_pct"], S=c["S"], rmax=c["rmax"], lag=0, trace_cap=0),
                (1, 2, 3, 4), (1, 2))
    shape_sweep("stream",
                lambda: hm.Stream(W=1, theta_pct=45, S=c["S"], rmax=c["rmax"], lag=c["lag"], trace_cap=0),
                (1, 2), (2, 4, 6, 8, 12, 16))   # launches that may wait take at most 2 per CU
    del arenas, a0

    # ---- Figure 5: degenerate + uniform mixture, d = 0..100 %
    n = 64 * MIB
    fig5 = {}
    ds = [0, 5, 10, 20, 30, 40, 45, 50, 60, 70, 80, 90, 100]
    for d in ds:
        x = G.mixture_bytes(n, d / 100.0, 127, G.rng(6, d))
        xd = torch.from_numpy(x).to(dev)
        h = np.bincount(x, minlength=256)     # the pattern a stream would derive from this data
        kernels = {"wavehist": (hm.MODE_WAVEHIST, None), "waveagg": (hm.MODE_WAVEAGG, None),
                   "ahist_paper960": (hm.MODE_AHIST, hm.pattern_init(hm.PAT_PAPER960)),
                   "ahist_ruleP_960_8": (hm.MODE_AHIST, rule_p_host(h, 960, 8)),
                   "ahist_flat32": (hm.MODE_AUTO, None)}
        row = {}
        for name, (mode, pat) in kernels.items():
            ms = timed(torch, lambda: hm.hist_u8(xd, out, mode=mode, pattern=pat), 10)
            row[name] = round(n / ms / 1e6, 1)
        fig5[d] = row
        log("fig5 d=%d" % d, row)
    result["sweeps"]["fig5_GBps"] = fig5

    def crossover(a, b):
        """Smallest d at which kernel a is faster than kernel b (100 if never)."""
        for d in ds:
            if fig5[d][a] > fig5[d][b]:
                return d
        return 100
    result["theta_crossover_pct"] = {
        "ruleP_960_vs_wavehist": crossover("ahist_ruleP_960_8", "wavehist"),
        "flat32_vs_wavehist": crossover("ahist_flat32", "wavehist"),
        "paper960_vs_wavehist": crossover("ahist_paper960", "wavehist"),
    }
    log("crossovers", result["theta_crossover_pct"])
    result["written"] = time.strftime("%Y-%m-%d %H:%M:%S")
    with open(args.out, "w") as f:
        json.dump(result, f, indent=1)
        f.write("\n")
    log("wrote", args.out)


if __name__ == "__main__":
    main()
