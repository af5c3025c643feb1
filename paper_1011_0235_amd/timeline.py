"""Per-step breakdown of one launch, in the manner of the paper's Table 1 (Sec. III.A).

Runs workloads through the diagnostic library libhistmi_timeline.so (the same kernel with
per-workgroup event timestamps, include/histmi_timeline.h) and reports, for one launch of
each, when the steps of the path end across the grid:

  start   kernel arguments read, counting table cleared, segment set up (pattern / decision)
  count   16-byte loads and one LDS add per byte
  flush   sub-bins summed per value, added into the partial copies
  merge   the finalizer's sum of the copies, the histogram written (and the stream epilogue)

with the cumulative throughput of the launch up to the end of each step, next to the plain
streaming read of the same bytes (hist_read_probe), which stands in for Table 1's first row.

    python -m paper_1011_0235_amd.timeline [--json]

Must run in a fresh process: it loads the diagnostic library in place of libhistmi.so.
"""

import ctypes
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_TIMELINE = os.path.join(HERE, "libhistmi_timeline.so")

PHASE = {0: "entry", 2: "set up", 3: "tile counted", 4: "flushed", 5: "finalizer start", 6: "merged",
         7: "finalizer done", 8: "exit", 9: "flush start", 10: "table summed", 11: "atomics issued"}


def _events(buf, wgs, per):
    """Per workgroup: list of (phase, segment, time in us) of the recorded events."""
    b = buf.reshape(wgs, per)
    out = []
    for g in range(wgs):
        row = b[g]
        row = row[row != 0]
        if row.size:
            out.append([(int(x >> 56), int((x >> 40) & 0xFFFF), int(x & ((1 << 40) - 1)) / 100.0) for x in row])
    return out


def analyse(events, nbytes):
    t0 = min(e[0][2] for e in events)
    last = {}
    first_setup = 0.0   # the latest workgroup's first segment set up
    per_wg = {"start": [], "count": [], "flush": []}
    for ev in events:
        times = {}
        for ph, _, t in ev:
            times.setdefault(ph, []).append(t - t0)
            last[ph] = max(last.get(ph, 0.0), t - t0)
        if 2 in times:
            first_setup = max(first_setup, min(times[2]))
        if 0 in times and 2 in times:
            per_wg["start"].append(min(times[2]) - min(times[0]))
        if 2 in times and 3 in times:
            per_wg["count"].append(max(times[3]) - min(times[2]))
        if 3 in times and 4 in times:
            per_wg["flush"].append(max(times[4]) - max(times[3]))
    span = max(t - t0 for ev in events for _, _, t in ev)
    steps = [("start", "arguments read, table cleared, first segment set up", first_setup),
             ("count", "16-byte loads, one LDS add per byte", last.get(3, 0.0)),
             ("flush", "sub-bins summed, added into the partial copies", last.get(4, 0.0)),
             ("merge", "copies summed, histogram written (stream epilogue)", max(last.get(7, 0.0), span))]
    rows = []
    for name, what, end in steps:
        rows.append({"step": name, "what": what, "ends_us": round(end, 2),
                     "cumulative_GBps": round(nbytes / (end * 1e-6) / 1e9, 1) if end > 0 else None})
    med = {k: (round(float(np.median(v)), 2), round(float(np.percentile(v, 90)), 2)) for k, v in per_wg.items() if v}
    return {"workgroups": len(events), "span_us": round(span, 2), "steps": rows,
            "per_workgroup_p50_p90_us": med}


def main(argv):
    import torch   # the library binds to PyTorch's HIP runtime
    from paper_1011_0235_amd import _lib as L
    lib = L.load(LIB_TIMELINE)
    for f in (lib.hist_timeline_shape, lib.hist_timeline_read, lib.hist_timeline_reset):
        f.restype = ctypes.c_int
    import paper_1011_0235_amd as hm
    sys.path.insert(0, ROOT)
    import synthgen as G
    wgs, per = ctypes.c_uint32(), ctypes.c_uint32()
    assert lib.hist_timeline_shape(ctypes.byref(wgs), ctypes.byref(per)) == 0
    wgs, per = wgs.value, per.value
    buf = np.zeros(wgs * per, dtype=np.uint64)
    s = torch.cuda.current_stream()

    def capture(fn):
        torch.cuda.synchronize()
        assert lib.hist_timeline_reset() == 0
        fn()
        torch.cuda.synchronize()
        assert lib.hist_timeline_read(buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                      ctypes.c_size_t(buf.nbytes)) == 0
        return _events(buf, wgs, per)

    out = {}
    # Table 2's 64 MiB slice of random bytes, one hist_u8 launch; its read probe for row 1
    x = torch.from_numpy(G.table2_input("random")).cuda()
    o = torch.zeros(256, dtype=torch.int32, device="cuda")
    for _ in range(5):
        hm.hist_u8(x, o, stream=s)
    ev = capture(lambda: hm.hist_u8(x, o, stream=s))
    row = analyse(ev, x.numel())
    # the plain streaming read (Table 1's first row), over 1 GiB so that its own start and
    # its final sum do not dominate, at the bench's best grid
    sums = torch.zeros(1, dtype=torch.int64, device="cuda")
    big = torch.empty(1 << 30, dtype=torch.uint8, device="cuda").random_(0, 256)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        hm.read_probe(big, sums, workgroups=512, stream=s)
    e0.record(s)
    for _ in range(10):
        hm.read_probe(big, sums, workgroups=512, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    gbps = big.numel() / (ms * 1e-3) / 1e9
    row["read_probe"] = {"GBps": round(gbps, 1), "us_for_these_bytes": round(x.numel() / gbps / 1e3, 2)}
    del big
    row["counts_sum_to_n"] = int(o.cpu().numpy().astype(np.int64).sum()) == x.numel()
    out["hist_u8_64MiB_random"] = row
    # one 1 MiB image
    x1 = torch.from_numpy(G.image_1mib()).cuda()
    for _ in range(5):
        hm.hist_u8(x1, o, stream=s)
    out["hist_u8_1MiB"] = analyse(capture(lambda: hm.hist_u8(x1, o, stream=s)), x1.numel())
    # the single stream, one 66 x 4 MiB push alone (decisions known on the host)
    chunks = G.stream_chunks(4 << 20)
    arena = torch.from_numpy(np.concatenate(chunks)).cuda()
    bufs = [(int(arena.data_ptr()) + k * (4 << 20), 4 << 20) for k in range(len(chunks))]
    outs = torch.zeros((len(chunks), 256), dtype=torch.int32, device="cuda")
    st = hm.Stream(W=1, theta_pct=0, S=8192, rmax=32, lag=0, trace_cap=0)
    for _ in range(4):
        st.push_many(bufs, d_out=outs, stream=s)
    out["stream_push_66x4MiB"] = analyse(capture(lambda: st.push_many(bufs, d_out=outs, stream=s)), arena.numel())
    st.close()
    if "--json" in argv:
        print(json.dumps(out))
        return 0
    for name, r in out.items():
        print("%s: %d workgroups, span %.2f us%s" % (name, r["workgroups"], r["span_us"],
                                                     "; a plain streaming read of 1 GiB runs at %.1f GB/s, "
                                                     "%.2f us for these bytes" % (r["read_probe"]["GBps"],
                                                                                  r["read_probe"]["us_for_these_bytes"])
                                                     if "read_probe" in r else ""))
        print("| step | what | ends at (us) | cumulative GB/s |")
        print("|---|---|---|---|")
        for st_ in r["steps"]:
            print("| %s | %s | %.2f | %s |" % (st_["step"], st_["what"], st_["ends_us"], st_["cumulative_GBps"]))
        print("per workgroup (p50, p90 us):", r["per_workgroup_p50_p90_us"])
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
