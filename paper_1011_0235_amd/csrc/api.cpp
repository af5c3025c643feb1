// C ABI of libhistmi: argument checks, launch planning, library-owned scratch, streams,
// batches and batch graphs.  Every histogram is computed by the HIP kernels in kernels.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "histmi.h"
#include "histmi_dev.h"
#include "runtime.h"

namespace histmi {
namespace rt {

// Defaults from the gfx950 probes: the lane-cyclic table streams best with 2 workgroups of
// 4 wavefronts per CU and 4 loads in flight per lane.
Tune g_tune[kFamilies] = {{4, 256, 4, 6}, {2, 256, 4, 6}, {2, 256, 4, 6}, {4, 256, 4, 6}, {3, 1024, 4, 4},
                          {2, 1024, 4, 2}};
uint32_t g_single_copies = 16;   // partial copies for a launch with one large segment
// bounded waits: polls of a decision tag (each about 0.3 us apart, about 1.2 s in all) and
// re-reads of a segment's partial copies before they give up
constexpr uint32_t kDefaultWaitPolls = 1u << 22;
constexpr uint32_t kDefaultMergePolls = 1u << 20;
static uint32_t g_wait_polls = kDefaultWaitPolls;
static uint32_t g_merge_polls = kDefaultMergePolls;

static std::mutex g_mu;
static std::unordered_map<int, DevCtx *> g_dev;

hist_status_t get_dev(DevCtx **out) {
  int dev = 0;
  TRY_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_dev.find(dev);
  if (it != g_dev.end()) {
    *out = it->second;
    return HIST_OK;
  }
  hipDeviceProp_t pr;
  TRY_HIP(hipGetDeviceProperties(&pr, dev));
  if (std::strncmp(pr.gcnArchName, "gfx950", 6) != 0) return HIST_ENOTSUP;
  DevCtx *d = new DevCtx();
  d->dev = dev;
  d->cus = pr.multiProcessorCount;
  d->lds_cu = pr.maxSharedMemoryPerMultiProcessor ? pr.maxSharedMemoryPerMultiProcessor : pr.sharedMemPerBlock;
  if (hipMalloc(&d->diag, 64 * sizeof(uint32_t)) != hipSuccess) {
    delete d;
    return HIST_ENOMEM;
  }
  if (hipMemset(d->diag, 0, 64 * sizeof(uint32_t)) != hipSuccess) {
    (void)hipFree(d->diag);
    delete d;
    return HIST_EDEVICE;
  }
  // allow dynamic LDS up to the CU's size; launches that need less work either way
  if (set_kernel_attrs((uint32_t)(d->lds_cu - kStaticLdsReserve)) != hipSuccess) (void)hipGetLastError();
  g_dev[dev] = d;
  *out = d;
  return HIST_OK;
}

// Grow-only device buffer; the old one is released after `s` drains.  New memory is zeroed on `s`.
template <typename T>
static hist_status_t ensure(T **p, size_t *cap, size_t need, hipStream_t s, bool zero) {
  if (need <= *cap && *p) return HIST_OK;
  const size_t ncap = std::max<size_t>(need, *cap * 2);
  if (*p) {
    TRY_HIP(hipStreamSynchronize(s));
    TRY_HIP(hipFree(*p));
    *p = nullptr;
    *cap = 0;
  }
  if (hipMalloc(reinterpret_cast<void **>(p), ncap * sizeof(T)) != hipSuccess) return HIST_ENOMEM;
  if (zero) TRY_HIP(hipMemsetAsync(*p, 0, ncap * sizeof(T), s));
  *cap = ncap;
  return HIST_OK;
}

hist_status_t alloc_scratch(Scratch *sc, size_t nseg, uint32_t copies, size_t desc_bytes, hipStream_t s) {
  TRY(ensure(&sc->ctr, &sc->ctr_cap, 64, s, true));
  TRY(ensure(&sc->seg_done, &sc->seg_cap, std::max<size_t>(nseg, 1), s, true));
  TRY(ensure(&sc->partial, &sc->partial_cap, std::max<size_t>(nseg, 1) * copies * 256, s, true));
  if (desc_bytes) {
    if (desc_bytes > sc->desc_cap) TRY(ensure(&sc->desc_buf, &sc->desc_cap, desc_bytes, s, false));
    sc->desc = sc->desc_buf;
    sc->cur = -1;
  }
  return HIST_OK;
}

void free_scratch(Scratch *sc) {
  if (sc->ctr) (void)hipFree(sc->ctr);
  if (sc->seg_done) (void)hipFree(sc->seg_done);
  if (sc->partial) (void)hipFree(sc->partial);
  if (sc->desc_buf) (void)hipFree(sc->desc_buf);
  for (auto &e : sc->cache)
    if (e.dev) (void)hipFree(e.dev);
  for (int k = 0; k < 2; ++k) {
    if (sc->stage[k]) (void)hipHostFree(sc->stage[k]);
    if (sc->ev[k]) (void)hipEventDestroy(sc->ev[k]);
  }
  *sc = Scratch();
}

hist_status_t get_scratch(DevCtx *d, hipStream_t s, size_t nseg, uint32_t copies, size_t desc_bytes,
                          Scratch **out) {
  Scratch *sc;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = d->scratch.find(s);
    if (it == d->scratch.end()) {
      sc = new Scratch();
      d->scratch[s] = sc;
    } else {
      sc = it->second;
    }
  }
  TRY(alloc_scratch(sc, nseg, copies, desc_bytes, s));
  *out = sc;
  return HIST_OK;
}

// Make the descriptors `host` available on the device and point sc->desc at them.  A set
// identical to one of the last few uploaded is reused as is; otherwise the least recently
// used cache entry is refilled through pinned staging (two buffers, each reused only after
// its previous copy finished).  The refill is a copy on `s`, the only HIP stream whose
// launches read this Scratch, so it runs after every launch that read the old contents.
hist_status_t upload_desc(Scratch *sc, const void *host, size_t bytes, hipStream_t s) {
  ++sc->tick;
  for (int i = 0; i < 4; ++i) {
    Scratch::Cached &e = sc->cache[i];
    if (e.dev && e.blob.size() == bytes && std::memcmp(e.blob.data(), host, bytes) == 0) {
      e.used = sc->tick;
      sc->desc = e.dev;
      sc->cur = i;
      return HIST_OK;
    }
  }
  int vi = 0;
  for (int i = 1; i < 4; ++i)
    if (sc->cache[i].used < sc->cache[vi].used) vi = i;
  Scratch::Cached *victim = &sc->cache[vi];
  if (victim->cap < bytes) {
    if (victim->dev) {
      TRY_HIP(hipStreamSynchronize(s));   // launches still reading the old buffer are done
      TRY_HIP(hipFree(victim->dev));
    }
    victim->dev = nullptr;
    victim->cap = 0;
    victim->blob.clear();
    const size_t cap = std::max<size_t>(bytes, 1 << 16);
    if (hipMalloc(&victim->dev, cap) != hipSuccess) return HIST_ENOMEM;
    victim->cap = cap;
  }
  const int k = sc->turn;
  sc->turn ^= 1;
  if (sc->ev[k]) TRY_HIP(hipEventSynchronize(sc->ev[k]));
  else TRY_HIP(hipEventCreateWithFlags(&sc->ev[k], hipEventDisableTiming));
  if (sc->stage_cap[k] < bytes) {
    if (sc->stage[k]) TRY_HIP(hipHostFree(sc->stage[k]));
    sc->stage[k] = nullptr;
    sc->stage_cap[k] = 0;
    const size_t cap = std::max<size_t>(bytes, 1 << 16);
    if (hipHostMalloc(reinterpret_cast<void **>(&sc->stage[k]), cap, hipHostMallocDefault) != hipSuccess)
      return HIST_ENOMEM;
    sc->stage_cap[k] = cap;
  }
  std::memcpy(sc->stage[k], host, bytes);
  TRY_HIP(hipMemcpyAsync(victim->dev, sc->stage[k], bytes, hipMemcpyHostToDevice, s));
  TRY_HIP(hipEventRecord(sc->ev[k], s));
  victim->blob.assign(static_cast<const uint8_t *>(host), static_cast<const uint8_t *>(host) + bytes);
  victim->used = sc->tick;
  sc->desc = victim->dev;
  sc->cur = vi;
  return HIST_OK;
}

hist_status_t reserve_scratch(Scratch *sc, size_t nseg, uint32_t copies, size_t desc_bytes, hipStream_t s) {
  TRY(alloc_scratch(sc, nseg, copies, 0, s));
  const size_t cap = std::max<size_t>(desc_bytes, 1 << 16);   // upload_desc's smallest buffers
  for (int k = 0; k < 2; ++k) {
    if (!sc->ev[k]) TRY_HIP(hipEventCreateWithFlags(&sc->ev[k], hipEventDisableTiming));
    if (sc->stage_cap[k] < cap) {
      if (sc->ev[k]) TRY_HIP(hipEventSynchronize(sc->ev[k]));
      if (sc->stage[k]) TRY_HIP(hipHostFree(sc->stage[k]));
      sc->stage[k] = nullptr;
      sc->stage_cap[k] = 0;
      if (hipHostMalloc(reinterpret_cast<void **>(&sc->stage[k]), cap, hipHostMallocDefault) != hipSuccess)
        return HIST_ENOMEM;
      sc->stage_cap[k] = cap;
    }
  }
  for (Scratch::Cached &e : sc->cache) {
    if (e.cap >= cap) continue;
    if (e.dev) {
      TRY_HIP(hipStreamSynchronize(s));   // launches still reading the old buffer are done
      TRY_HIP(hipFree(e.dev));
    }
    e.dev = nullptr;
    e.cap = 0;
    e.blob.clear();
    if (hipMalloc(&e.dev, cap) != hipSuccess) return HIST_ENOMEM;
    e.cap = cap;
  }
  return HIST_OK;
}

bool pattern_ok(const hist_pattern_t *p) {
  const uint32_t S = p->total_S, rmax = p->rmax;
  if (!is_pow2(rmax) || rmax > HIST_RMAX_MAX || S < 1 || S > HIST_S_MAX) return false;
  std::vector<uint8_t> used(S, 0);
  for (int v = 0; v < 256; ++v) {
    const uint32_t w = p->word[v];
    if (w >> 24) return false;
    const uint32_t lg = (w >> 16) & 0xFF, base = w & 0xFFFF;
    if (lg > 6 || (1u << lg) > rmax) return false;
    const uint32_t r = 1u << lg;
    if (base + r > S) return false;
    for (uint32_t i = base; i < base + r; ++i) {
      if (used[i]) return false;
      used[i] = 1;
    }
  }
  return true;
}

void init_params(Params *P) {
  std::memset(P, 0, sizeof(*P));
  P->seg0.chunk = -1;
  P->wait_polls = g_wait_polls;
  P->merge_polls = g_merge_polls;
}

// LDS layout: counting table of `table_words` at word 0, then the lookup table.
static void set_lds(Params *P, uint32_t table_words, bool lookup, uint32_t rr_lg) {
  P->table_words = (std::max<uint32_t>(table_words, kWaves * 256) + 3u) & ~3u;
  P->look_off = P->table_words;
  P->look_rr_lg = rr_lg;
  P->look_words = lookup ? (256u << rr_lg) : 0u;
}

hist_status_t select_kind(hist_mode_t mode, const hist_pattern_t *h_pat, Params *P) {
  uint32_t table = kWaves * 256;
  bool lookup = false;
  uint32_t rr_lg = 5;
  if (mode == HIST_MODE_WAVEHIST) {
    P->kind = KIND_WAVE;
  } else if (mode == HIST_MODE_WAVEAGG) {
    P->kind = KIND_WAVE_AGG;
  } else if (mode == HIST_MODE_AUTO) {
    P->kind = KIND_UNIFORM;
    P->uni_lg = log2u(HIST_AUTO_FLAT_R);
    table = 256u << P->uni_lg;
  } else if (mode == HIST_MODE_AHIST) {
    if (!h_pat) {
      P->kind = KIND_UNIFORM;   // identity pattern: r = 1, base = value
      P->uni_lg = 0;
      table = 256;
    } else {
      if (!pattern_ok(h_pat)) return HIST_EINVAL;
      const uint32_t lg0 = (h_pat->word[0] >> 16) & 0xFF;
      bool uni = true;
      for (uint32_t v = 0; v < 256 && uni; ++v) uni = (h_pat->word[v] == ((v << lg0) | (lg0 << 16)));
      if (uni) {
        P->kind = KIND_UNIFORM;
        P->uni_lg = lg0;
        table = 256u << lg0;
      } else {
        P->kind = KIND_LOOKUP;
        P->pat_S = h_pat->total_S;
        for (int v = 0; v < 256; ++v) P->pat_words[v] = h_pat->word[v];
        rr_lg = h_pat->rmax > 32 ? 6 : 5;
        table = h_pat->total_S;
        lookup = true;
      }
    }
  } else {
    return HIST_EINVAL;
  }
  set_lds(P, table, lookup, rr_lg);
  return HIST_OK;
}

void stream_layout(uint32_t S, uint32_t rmax, hist_mode_t mode, Params *P) {
  const bool saturated = 256u * rmax <= S;   // rule P then always gives the uniform pattern
  P->forced = mode == HIST_MODE_AUTO ? 0u : (uint32_t)mode;
  P->pat_S = S;
  P->kind = KIND_WAVE;
  set_lds(P, std::max<uint32_t>(S, 256u * rmax), !saturated, rmax > 32 ? 6 : 5);
}

uint32_t lds_bytes(const Params &P) { return (P.table_words + P.look_words) * 4u + ctl_bytes(); }

// Workgroups per CU: the family's tuned value, capped by what fits.
// Workgroups of the counting kernel that fit on one CU with `lds` bytes of dynamic LDS.
uint32_t resident_per_cu(uint32_t lds) {
  static std::mutex mu;
  static std::unordered_map<uint32_t, int> cache;   // dynamic LDS bytes -> resident workgroups per CU
  int occ = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(lds);
    if (it != cache.end()) occ = it->second;
  }
  if (occ == 0) {
    if (occupancy(lds, &occ) != hipSuccess || occ < 1) occ = 1;
    std::lock_guard<std::mutex> lk(mu);
    cache[lds] = occ;
  }
  return (uint32_t)occ;
}

uint32_t blocks_per_cu(uint32_t family, uint32_t lds) {
  return std::max<uint32_t>(1, std::min<uint32_t>(g_tune[family].bpc, resident_per_cu(lds)));
}

hist_status_t run_single(DevCtx *d, Params &P, hipStream_t s, Scratch *own, hipEvent_t done) {
  const uint64_t n = P.seg0.size;
  const uint32_t fam = P.st ? (uint32_t)KIND_UNIFORM : P.kind;
  const uint32_t lds = lds_bytes(P);
  const uint32_t G = (uint32_t)d->cus * blocks_per_cu(fam, lds);
  // one workgroup per 16 KiB of the buffer, at most the whole grid (every workgroup strides
  // over the buffer; the last one finalizes)
  const uint32_t ntiles = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(G, ceil_div(n, 16384)));
  // one partial copy per 8 workgroups, at most 16: the merge reads fewer copies and the
  // flush's atomics still spread (1 MiB, 64 workgroups: 5.5 us a call with 8 copies, 5.8-6.0
  // with 16, 6.6 with 4; larger launches take 16 either way)
  const uint32_t copies = std::min<uint32_t>(g_single_copies, pow2ceil32(std::max<uint32_t>(1, ntiles / 8)));
  Scratch *sc = own;
  if (!sc) TRY(get_scratch(d, s, 1, copies, 0, &sc));
  else TRY(alloc_scratch(sc, 1, copies, 0, s));
  P.seg0.tile0 = 0;
  P.seg0.ntiles = ntiles;
  P.nseg = 1;
  P.single = 1;
  P.ntiles = ntiles;
  P.dynamic = 0;
  P.clog2 = log2u(copies);
  P.ctr = sc->ctr;
  P.seg_done = sc->seg_done;
  P.partial = sc->partial;
  P.diag = d->diag;
  const LaunchShape sh{ntiles, lds, 4};
  return dev_err(launch_hist(P, sh, s, done));
}

hist_status_t run_multi(DevCtx *d, Params &P, const MultiPlan &mp, uint32_t copies, hipStream_t s, Scratch *own,
                        bool dynamic, bool upload, hipEvent_t done, const uint8_t *in_place) {
  Scratch *sc = own;
  if (!sc) TRY(get_scratch(d, s, mp.nseg, copies, 0, &sc));
  else TRY(alloc_scratch(sc, mp.nseg, copies, (upload || in_place) ? 0 : mp.blob.size(), s));
  if (upload && !in_place) TRY(upload_desc(sc, mp.blob.data(), mp.blob.size(), s));
  const uint8_t *desc = in_place ? in_place : sc->desc;
  P.segs = reinterpret_cast<const SegDesc *>(desc);
  P.recs = reinterpret_cast<const TileRec *>(desc + mp.seg_bytes);
  P.bounds = reinterpret_cast<const uint32_t *>(desc + mp.seg_bytes + mp.rec_bytes);
  P.starts = mp.start_off ? reinterpret_cast<const WgStart *>(desc + mp.start_off) : nullptr;
  P.nseg = mp.nseg;
  P.single = 0;
  P.ntiles = mp.ntiles;
  P.dynamic = dynamic ? 1u : 0u;
  P.clog2 = log2u(copies);
  P.ctr = sc->ctr;
  P.seg_done = sc->seg_done;
  P.partial = sc->partial;
  P.diag = d->diag;
  const LaunchShape sh{mp.grid, lds_bytes(P), 4};
  return dev_err(launch_hist(P, sh, s, done));
}

hist_status_t stream_state_alloc(uint32_t count, uint32_t W, uint32_t theta, uint32_t S, uint32_t rmax, uint32_t lag,
                                 uint32_t nslot, uint32_t trace_cap, uint32_t alarm_pct, StreamAlloc *sa) {
  const size_t tc = std::max<uint32_t>(trace_cap, 1);
  // W > 1 or alarms on: chunks are sequenced in order from a ring of recent histograms.
  // Chunk j's histogram is needed until chunk j + W is sequenced.  The ring may not rely on
  // chunks waiting for their decisions (a wait that gives up lets its chunk run and write
  // its entry anyway), only on how many chunks can be in flight: a workgroup that holds the
  // sequencer belongs to a running launch X, so at most launches X and X + 1 write entries
  // (a push waits for the launch two before it), while the oldest entry the holder can
  // still read belongs to launch X - 2 (every earlier chunk was present, and so taken in
  // order, before X - 1 ended), less the W chunks of the window before it.  Each launch
  // holds at most kMaxChunksPerLaunch chunks, so W + 4 kMaxChunksPerLaunch slots suffice;
  // lag + 1 more are kept as a margin.
  const uint32_t R = (W > 1 || alarm_pct > 0) ? W + lag + 1 + 4 * kMaxChunksPerLaunch : 1;
  sa->R = R;
  bool ok = hipMalloc(&sa->d_st, (size_t)count * sizeof(StreamDev)) == hipSuccess &&
            hipMalloc(&sa->d_ring, (size_t)count * R * 257 * 8) == hipSuccess &&
            hipMalloc(&sa->d_slots, (size_t)count * nslot * sizeof(Decision)) == hipSuccess &&
            hipMalloc(&sa->d_mode_trace, (size_t)count * tc * 2) == hipSuccess &&
            hipMalloc(&sa->d_pat_trace, (size_t)count * tc * 256 * 4) == hipSuccess &&
            hipMalloc(&sa->d_time_trace, (size_t)count * tc * 3 * 8) == hipSuccess;
  if (!ok) {
    stream_state_free(sa);
    return HIST_ENOMEM;
  }
  std::vector<StreamDev> h(count);
  for (uint32_t i = 0; i < count; ++i) {
    StreamDev &x = h[i];
    std::memset(&x, 0, sizeof(x));
    x.W = W;
    x.theta = theta;
    x.S = S;
    x.rmax = rmax;
    x.lag = lag;
    x.nslot = nslot;
    x.trace_cap = trace_cap;
    x.lookup_rr = rmax > 32 ? 64 : 32;
    x.R = R;
    x.alarm_pct = alarm_pct;
    x.ring = sa->d_ring + (size_t)i * R * 256;
    x.ring_n = sa->d_ring + (size_t)count * R * 256 + (size_t)i * R;
    x.slots = sa->d_slots + (size_t)i * nslot;
    x.mode_trace = sa->d_mode_trace + (size_t)i * tc;
    x.alarm_trace = sa->d_mode_trace + (size_t)count * tc + (size_t)i * tc;
    x.pat_trace = sa->d_pat_trace + (size_t)i * tc * 256;
  }
  ok = hipMemcpy(sa->d_st, h.data(), (size_t)count * sizeof(StreamDev), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemset(sa->d_ring, 0, (size_t)count * R * 257 * 8) == hipSuccess &&
       hipMemset(sa->d_slots, 0, (size_t)count * nslot * sizeof(Decision)) == hipSuccess &&
       hipMemset(sa->d_mode_trace, 0, (size_t)count * tc * 2) == hipSuccess &&
       hipMemset(sa->d_pat_trace, 0, (size_t)count * tc * 256 * 4) == hipSuccess &&
       hipMemset(sa->d_time_trace, 0xFF, (size_t)count * tc * 3 * 8) == hipSuccess;
  if (!ok) {
    stream_state_free(sa);
    return HIST_EDEVICE;
  }
  return HIST_OK;
}

void stream_state_free(StreamAlloc *sa) {
  if (sa->d_st) (void)hipFree(sa->d_st);
  if (sa->d_ring) (void)hipFree(sa->d_ring);
  if (sa->d_slots) (void)hipFree(sa->d_slots);
  if (sa->d_mode_trace) (void)hipFree(sa->d_mode_trace);
  if (sa->d_pat_trace) (void)hipFree(sa->d_pat_trace);
  if (sa->d_time_trace) (void)hipFree(sa->d_time_trace);
  *sa = StreamAlloc();
}

}  // namespace rt
}  // namespace histmi

using namespace histmi;
using namespace histmi::rt;

struct hist_stream {
  hist_stream_config_t cfg;
  uint32_t nslot = 0;
  uint64_t pushed = 0;
  StreamAlloc sa;
  // sizes of the last lag + 1 chunks (chunk k in slot k % (lag + 1)): with decisions that
  // depend on the chunk sizes only, the decision a chunk runs with is known on the host
  std::vector<uint64_t> recent;
  // Launches of one stream may run on different HIP streams and overlap; the device makes
  // each chunk wait for its decision.  At most two launches are in flight: before a launch,
  // the HIP stream waits for the launch two before it.  Slot i describes one of the last
  // two launches: the HIP stream it went to, and whether ev[i] has been recorded on that
  // HIP stream since (so that it completes with or after the launch).  Events are recorded
  // only when a launch on another HIP stream has to wait: an event packet between two
  // kernels costs the device a few microseconds, and a launch on the same HIP stream is
  // ordered anyway (two HIP streams used in turn never need one).
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ev_used[2] = {false, false};
  bool ev_rec[2] = {false, false};
  hipStream_t ev_on[2] = {nullptr, nullptr};
  uint32_t evi = 0;
  std::vector<hipStream_t> used;   // HIP streams with launches of this stream since the last read
  // Waiting for the launch two before splits the launches into two chains (odd and even);
  // chunks that wait for decisions tie the chains together on the device, but chunks whose
  // decisions the host knows do not, so one chain could run ahead of the other, further
  // than the decision ring holds.  Such streams therefore order a launch after every
  // earlier one once the chunks pushed since the last such point would pass
  // kMaxChunksPerLaunch: at most 2 x kMaxChunksPerLaunch chunks are ever in flight.
  uint64_t since_join = 0;
  // A window stream with the uniform switch and no change detection does not walk its window
  // in order (its chunks carry kUnwalked; the configuration fixes this for every launch):
  // nothing in a launch needs the window, so the device's copy of it falls behind until
  // window_rebuild_kernel sums it from the ring again, before a read.
  bool window_stale = false;
};

// Whether every decision is a function of the chunk sizes alone: a budget that gives every
// value rmax sub-bins (rule P's first case: the pattern is the uniform table whatever the
// histogram) and a switching test that fires for any non-empty window (theta or kappa 0).
// The decision after chunk j is then AHist if the window up to chunk j holds a byte, else
// the per-wavefront kernel, with the uniform table either way.
static bool decisions_uniform(const hist_stream_config_t &c) {
  if (256ull * c.rmax > c.S) return false;
  switch (c.criterion) {
  case HIST_CRIT_MAXBIN: return c.theta_pct == 0;
  case HIST_CRIT_COLLISION: return c.kappa_pct == 0;
  default: return c.theta_pct == 0 || c.kappa_pct == 0;
  }
}

// The host hands each chunk of a launch its decision (the chunk then starts without
// waiting; the device still publishes the same decisions) when the decisions are uniform as
// above.  Nothing in such a launch waits for the in-order walk of the window, so it runs on
// equal byte shares like a stream with W = 1.  A window stream without change detection does
// not walk at all (see hist_stream::window_stale); with change detection the walk follows
// the counting launch in a one-workgroup launch of its own (walk_kernel).  Before this, such
// pushes walked inside the counting launch: on dynamic tiles, so that a workgroup that walks
// for a while leaves no static share behind (W = 32, lag 31, change detection at 4 points:
// 2.87 TB/s), and pushes whose decisions all came from an earlier push waited on it on
// equal shares (W = 32, lag 65 without change detection: 4.96 TB/s).
static bool decisions_known(const hist_stream_config_t &c) { return decisions_uniform(c); }

// Make `s` wait for the launch in slot i, unless that launch went to `s` itself (then it is
// ordered before anything queued on `s` now).  Its event is recorded on its HIP stream now
// if it was not yet: that covers the launch and whatever was queued after it there.
static hist_status_t wait_slot(hist_stream *st, uint32_t i, hipStream_t s) {
  if (!st->ev_used[i] || st->ev_on[i] == s) return HIST_OK;
  if (!st->ev_rec[i]) {
    TRY_HIP(hipEventRecord(st->ev[i], st->ev_on[i]));
    st->ev_rec[i] = true;
  }
  TRY_HIP(hipStreamWaitEvent(s, st->ev[i], 0));
  return HIST_OK;
}
// Before a launch: wait for the launch two before it (at most two in flight), or, with
// `serialize`, for both earlier ones (no overlap; every earlier launch is then done, since
// each waited for the one two before it).
static hist_status_t stream_launch_begin(hist_stream *st, hipStream_t s, bool serialize) {
  TRY(wait_slot(st, st->evi, s));
  if (serialize) TRY(wait_slot(st, st->evi ^ 1u, s));
  return HIST_OK;
}
static void stream_launch_end(hist_stream *st, hipStream_t s) {
  st->ev_used[st->evi] = true;
  st->ev_rec[st->evi] = false;
  st->ev_on[st->evi] = s;
  st->evi ^= 1u;
  if (std::find(st->used.begin(), st->used.end(), s) == st->used.end()) st->used.push_back(s);
}
// Wait on the host for every launch of the stream (synchronous reads).
static hist_status_t stream_sync(hist_stream *st, hipStream_t s) {
  TRY_HIP(hipStreamSynchronize(s));
  for (hipStream_t u : st->used)
    if (u != s) TRY_HIP(hipStreamSynchronize(u));
  st->used.clear();
  return HIST_OK;
}

struct hist_batch_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  Scratch sc;
};

extern "C" {

const char *hist_strerror(hist_status_t e) {
  switch (e) {
    case HIST_OK: return "ok";
    case HIST_EINVAL: return "invalid argument";
    case HIST_ENOMEM: return "out of memory";
    case HIST_EOVERFLOW: return "count could overflow its output";
    case HIST_EBUSY: return "busy";
    case HIST_EDEVICE: return "HIP device error";
    case HIST_ENOTSUP: return "not supported on this device";
    case HIST_ETIMEDOUT: return "timed out";
    case HIST_ECANCELED: return "canceled";
  }
  return "unknown status";
}

hist_status_t hist_device_info(hist_device_info_t *info) {
  if (!info) return HIST_EINVAL;
  int dev = 0;
  TRY_HIP(hipGetDevice(&dev));
  hipDeviceProp_t pr;
  TRY_HIP(hipGetDeviceProperties(&pr, dev));
  std::memset(info, 0, sizeof(*info));
  info->device = dev;
  info->cu_count = pr.multiProcessorCount;
  info->clock_khz = pr.clockRate;
  info->lds_per_cu = pr.maxSharedMemoryPerMultiProcessor;
  info->hbm_bytes = pr.totalGlobalMem;
  std::snprintf(info->arch, sizeof(info->arch), "%s", pr.gcnArchName);
  return HIST_OK;
}

hist_status_t hist_pattern_init(hist_pattern_t *p, hist_pattern_kind_t kind, uint32_t S, uint32_t rmax) {
  (void)S;
  if (!p) return HIST_EINVAL;
  uint32_t r[256];
  if (kind == HIST_PAT_IDENTITY) {
    for (int v = 0; v < 256; ++v) r[v] = 1;
    p->rmax = 1;
  } else if (kind == HIST_PAT_PAPER960) {
    static const uint32_t runs[8] = {1, 2, 4, 8, 8, 4, 2, 1};
    for (int v = 0; v < 256; ++v) r[v] = runs[v / 32];
    p->rmax = 8;
  } else if (kind == HIST_PAT_FLAT) {
    if (!is_pow2(rmax) || rmax > HIST_RMAX_MAX) return HIST_EINVAL;
    for (int v = 0; v < 256; ++v) r[v] = rmax;
    p->rmax = rmax;
  } else {
    return HIST_EINVAL;
  }
  uint32_t base = 0;
  for (int v = 0; v < 256; ++v) {
    p->word[v] = base | (log2u(r[v]) << 16);
    base += r[v];
  }
  p->total_S = base;
  return HIST_OK;
}

hist_status_t hist_pattern_validate(const hist_pattern_t *p) {
  if (!p) return HIST_EINVAL;
  return pattern_ok(p) ? HIST_OK : HIST_EINVAL;
}

hist_status_t hist_pattern_update(const uint64_t *d_hist, uint32_t S, uint32_t rmax, hist_pattern_t *d_pat,
                                  void *stream) {
  if (!d_hist || !d_pat || S < 256 || S > HIST_S_MAX || !is_pow2(rmax) || rmax > HIST_RMAX_MAX) return HIST_EINVAL;
  DevCtx *d;
  TRY(get_dev(&d));
  return dev_err(launch_pattern_update(d_hist, S, rmax, d_pat, static_cast<hipStream_t>(stream)));
}

static hist_status_t hist_common(const void *d_in, size_t n, uint32_t *d_out, uint64_t *d_acc, hist_mode_t mode,
                                 const hist_pattern_t *h_pat, void *stream) {
  if (n && !d_in) return HIST_EINVAL;
  if (!mode_ok(mode)) return HIST_EINVAL;
  if (d_out && (uint64_t)n > kMaxSegBytes) return HIST_EOVERFLOW;
  Params P;
  init_params(&P);
  TRY(select_kind(mode, h_pat, &P));
  DevCtx *d;
  TRY(get_dev(&d));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (d_out) {
    P.seg0.ptr = static_cast<const uint8_t *>(d_in);
    P.seg0.size = n;
    P.seg0.out = d_out;
    return run_single(d, P, s);
  }
  // accumulate in pieces whose counts fit the 32-bit partials
  const uint64_t piece = 1ull << 31;
  uint64_t done = 0;
  do {
    const uint64_t m = std::min<uint64_t>(piece, (uint64_t)n - done);
    P.seg0.ptr = static_cast<const uint8_t *>(d_in) + done;
    P.seg0.size = m;
    P.seg0.acc = d_acc;
    TRY(run_single(d, P, s));
    done += m;
  } while (done < (uint64_t)n);
  return HIST_OK;
}

hist_status_t hist_u8(const void *d_in, size_t n, uint32_t *d_out, hist_mode_t mode, const hist_pattern_t *h_pat,
                      void *stream) {
  if (!d_out) return HIST_EINVAL;
  return hist_common(d_in, n, d_out, nullptr, mode, h_pat, stream);
}

hist_status_t hist_u8_u64(const void *d_in, size_t n, uint64_t *d_acc, hist_mode_t mode, const hist_pattern_t *h_pat,
                          void *stream) {
  if (!d_acc) return HIST_EINVAL;
  return hist_common(d_in, n, nullptr, d_acc, mode, h_pat, stream);
}

// ---------------------------------------------------------------- batches

static hist_status_t batch_prepare(const void *const *h_ptrs, const uint64_t *h_sizes, uint32_t n, uint32_t *d_out,
                                   hist_mode_t mode, const hist_pattern_t *h_pat, DevCtx **dout, Params *P,
                                   MultiPlan *mp, uint32_t *copies) {
  if (!h_ptrs || !h_sizes || !d_out) return HIST_EINVAL;
  if (!mode_ok(mode)) return HIST_EINVAL;
  init_params(P);
  TRY(select_kind(mode, h_pat, P));
  DevCtx *d;
  TRY(get_dev(&d));
  *dout = d;
  const uint32_t fam = P->kind;
  const uint32_t maxg = (uint32_t)d->cus * blocks_per_cu(fam, lds_bytes(*P));
  // tiles: at most the tuned size, and small enough that every workgroup gets several
  uint64_t total = 0;
  for (uint32_t j = 0; j < n; ++j) total += h_sizes[j];
  const uint64_t want = ceil_div(ceil_div(total, (uint64_t)maxg * g_tune[fam].tpw), 16384) * 16384;
  const uint64_t tile = std::max<uint64_t>(16384, std::min<uint64_t>((uint64_t)g_tune[fam].tile_kib * 1024, want));
  std::vector<SegDesc> segs(n);
  for (uint32_t j = 0; j < n; ++j) {
    std::memset(&segs[j], 0, sizeof(SegDesc));
    segs[j].ptr = static_cast<const uint8_t *>(h_ptrs[j]);
    segs[j].size = h_sizes[j];
    segs[j].out = d_out + (size_t)j * 256;
    segs[j].chunk = -1;
  }
  TRY(plan_split(segs, tile, maxg, mp));
  *copies = std::min<uint32_t>(64, pow2ceil32(std::max<uint32_t>(1, g_tune[fam].copies)));
  return HIST_OK;
}

hist_status_t hist_batch(const void *const *h_ptrs, const uint64_t *h_sizes, uint32_t n, uint32_t *d_out,
                         hist_mode_t mode, const hist_pattern_t *h_pat, void *stream) {
  if (n == 0) return HIST_OK;
  DevCtx *d = nullptr;
  Params P;
  MultiPlan mp;
  uint32_t copies = 1;
  TRY(batch_prepare(h_ptrs, h_sizes, n, d_out, mode, h_pat, &d, &P, &mp, &copies));
  return run_multi(d, P, mp, copies, static_cast<hipStream_t>(stream), nullptr, false, true);
}

hist_status_t hist_batch_graph_destroy(hist_batch_graph_t *g);

hist_status_t hist_batch_graph_create(hist_batch_graph_t **g, const void *const *h_ptrs, const uint64_t *h_sizes,
                                      uint32_t n, uint32_t *d_out, hist_mode_t mode, const hist_pattern_t *h_pat) {
  if (!g || n == 0) return HIST_EINVAL;
  DevCtx *d = nullptr;
  Params P;
  MultiPlan mp;
  uint32_t copies = 1;
  TRY(batch_prepare(h_ptrs, h_sizes, n, d_out, mode, h_pat, &d, &P, &mp, &copies));
  hist_batch_graph *bg = new hist_batch_graph();
  hipStream_t cs = nullptr;
  hist_status_t st = HIST_OK;
  do {
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) { st = HIST_EDEVICE; break; }
    // graph-owned scratch, zeroed and loaded before capture (no memset or copy nodes in the graph)
    if ((st = alloc_scratch(&bg->sc, n, copies, mp.blob.size(), cs)) != HIST_OK) break;
    if (hipMemcpyAsync(bg->sc.desc, mp.blob.data(), mp.blob.size(), hipMemcpyHostToDevice, cs) != hipSuccess ||
        hipStreamSynchronize(cs) != hipSuccess) { st = HIST_EDEVICE; break; }
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) { st = HIST_EDEVICE; break; }
    st = run_multi(d, P, mp, copies, cs, &bg->sc, false, false);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(cs, &graph);
    if (graph) bg->graph = graph;
    if (st != HIST_OK) break;
    if (ce != hipSuccess || !graph) { st = HIST_EDEVICE; break; }
    if (hipGraphInstantiate(&bg->exec, graph, nullptr, nullptr, 0) != hipSuccess) { st = HIST_EDEVICE; break; }
  } while (0);
  if (cs) (void)hipStreamDestroy(cs);
  if (st != HIST_OK) {
    hist_batch_graph_destroy(bg);
    return st;
  }
  *g = bg;
  return HIST_OK;
}

hist_status_t hist_batch_graph_launch(hist_batch_graph_t *g, void *stream) {
  if (!g || !g->exec) return HIST_EINVAL;
  return dev_err(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
}

hist_status_t hist_batch_graph_destroy(hist_batch_graph_t *g) {
  if (!g) return HIST_EINVAL;
  (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  free_scratch(&g->sc);
  delete g;
  return HIST_OK;
}

// ---------------------------------------------------------------- streams

hist_status_t hist_stream_destroy(hist_stream_t *st);

hist_status_t hist_stream_create(hist_stream_t **out, const hist_stream_config_t *cfg) {
  if (!out || !cfg) return HIST_EINVAL;
  const hist_stream_config_t c = *cfg;
  if (c.W < 1 || c.W > (1u << 16) || c.theta_pct > 100 || c.S < 256 || c.S > HIST_S_MAX || !is_pow2(c.rmax) ||
      c.rmax > HIST_RMAX_MAX || c.lag > 4096 || c.trace_cap > (1u << 22) || c.alarm_pct > 100 ||
      c.criterion > HIST_CRIT_BOTH || c.kappa_pct > 100)
    return HIST_EINVAL;
  DevCtx *d;
  TRY(get_dev(&d));
  hist_stream *st = new hist_stream();
  st->cfg = c;
  // no decision slot is reused while a chunk may still read it: the two launches that can be
  // in flight span at most 2 * kMaxChunksPerLaunch chunks, plus the lag + 1 decisions made
  // before them
  st->nslot = c.lag + 2 + 2 * kMaxChunksPerLaunch;
  st->recent.assign((size_t)c.lag + c.W, 0);   // sizes of the last lag + W chunks
  hist_status_t r =
      stream_state_alloc(1, c.W, c.theta_pct, c.S, c.rmax, c.lag, st->nslot, c.trace_cap, c.alarm_pct, &st->sa);
  for (int i = 0; i < 2 && r == HIST_OK; ++i)
    if (hipEventCreateWithFlags(&st->ev[i], hipEventDisableTiming) != hipSuccess) r = HIST_EDEVICE;
  if (r != HIST_OK) {
    for (int i = 0; i < 2; ++i)
      if (st->ev[i]) (void)hipEventDestroy(st->ev[i]);
    stream_state_free(&st->sa);
    delete st;
    return r;
  }
  *out = st;
  return HIST_OK;
}

// The stream's state and the constants a chunk needs before it can start (copied into the
// launch's parameters so that the device reads only the decision's tag).
static void stream_params(const hist_stream *st, Params *P) {
  P->st = st->sa.d_st;
  P->ordered = 1;
  P->slots = st->sa.d_slots;
  P->lag = st->cfg.lag;
  P->nslot = st->nslot;
  P->W = st->cfg.W;
  P->alarm_pct = st->cfg.alarm_pct;
  P->criterion = st->cfg.criterion;
  P->kappa = st->cfg.kappa_pct;
  P->theta = st->cfg.theta_pct;
  P->S = st->cfg.S;
  P->rmax = st->cfg.rmax;
  P->R = st->sa.R;
  P->trace_cap = st->cfg.trace_cap;
  P->time_trace = st->sa.d_time_trace;
}

hist_status_t hist_stream_push(hist_stream_t *st, const void *d_chunk, size_t n, hist_mode_t mode, uint32_t *d_out_k,
                               void *stream) {
  // one chunk is a one-segment launch of the tiled kernel: a launch whose chunks may wait
  // for decisions hands its tiles out dynamically, so it completes with however many of its
  // workgroups are resident -- which overlapping launches on other HIP streams rely on (a
  // launch with every decision known waits for nothing and plans its tiles statically)
  if (!st || (n && !d_chunk) || !mode_ok(mode)) return HIST_EINVAL;
  if ((uint64_t)n > kMaxSegBytes) return HIST_EOVERFLOW;
  const void *p = d_chunk;
  const uint64_t size = n;
  return hist_stream_push_many(st, &p, &size, 1, mode, d_out_k, stream);
}

hist_status_t hist_stream_push_many(hist_stream_t *st, const void *const *h_ptrs, const uint64_t *h_sizes,
                                    uint32_t count, hist_mode_t mode, uint32_t *d_out, void *stream) {
  if (!st || !mode_ok(mode)) return HIST_EINVAL;
  if (count == 0) return HIST_OK;
  if (!h_ptrs || !h_sizes) return HIST_EINVAL;
  for (uint32_t j = 0; j < count; ++j) {
    if (h_sizes[j] > kMaxSegBytes) return HIST_EOVERFLOW;
    if (h_sizes[j] && !h_ptrs[j]) return HIST_EINVAL;
  }
  DevCtx *d;
  TRY(get_dev(&d));
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (uint32_t first = 0; first < count; first += kMaxChunksPerLaunch) {
    const uint32_t m = std::min<uint32_t>(kMaxChunksPerLaunch, count - first);
    Params P;
    init_params(&P);
    stream_layout(st->cfg.S, st->cfg.rmax, mode, &P);
    stream_params(st, &P);
    P.chunk_base = st->pushed;
    const bool known = decisions_known(st->cfg);
    const bool sequenced = st->cfg.W > 1 || st->cfg.alarm_pct != 0;
    const bool unwalked = known && sequenced && st->cfg.alarm_pct == 0;
    const bool walk_after = known && st->cfg.alarm_pct != 0;
    const uint32_t fam = known ? kFamStreamKnown : kFamStream;
    // Chunks that wait for decisions spin on their CU.  Two launches of the stream may be in
    // flight, and the hardware dispatches both at once: if they could not all be resident
    // together, the later launch's waiting workgroups could hold the CUs that the earlier
    // launch -- whose chunks they wait for -- needs.  So a launch that may wait takes at most
    // half of what a CU holds; where a CU holds only one, launches of the stream do not
    // overlap.
    const uint32_t occ = resident_per_cu(lds_bytes(P));
    const uint32_t bpc = known ? blocks_per_cu(fam, lds_bytes(P))
                               : std::max<uint32_t>(1, std::min(blocks_per_cu(fam, lds_bytes(P)), occ / 2));
    const bool serialize = !known && occ < 2;
    const uint32_t maxg = (uint32_t)d->cus * bpc;
    // the largest tile; launches that may wait cut tiles small enough that the lag + 1 chunks
    // which may run at once still fill the grid
    uint64_t tile = (uint64_t)g_tune[fam].tile_kib * 1024;
    if (!known) {
      uint64_t total = 0;
      for (uint32_t j = 0; j < m; ++j) total += h_sizes[first + j];
      const uint64_t per_chunk = std::max<uint64_t>(1, total / m);
      const uint64_t inflight = std::min<uint32_t>(st->cfg.lag + 1, m);
      const uint64_t fill = known ? ~0ull : ceil_div(per_chunk * inflight, maxg);   // lag + 1 chunks cover the grid
      const uint64_t several = ceil_div(total, (uint64_t)maxg * g_tune[fam].tpw);   // tiles per workgroup
      tile = std::min<uint64_t>(tile, std::max<uint64_t>(16384, ceil_div(std::min(fill, several), 16384) * 16384));
    }
    std::vector<SegDesc> segs(m);
    const uint32_t ring = st->cfg.lag + st->cfg.W;
    const uint32_t lgmax = log2u(st->cfg.rmax);
    // known decisions: chunk k runs with the decision made after chunk src = k - 1 - lag,
    // AHist with the uniform table iff one of chunks src - W + 1 .. src holds a byte;
    // nz[q - lo] counts the non-empty chunks in [lo, q)
    const int64_t k0 = (int64_t)st->pushed, W = (int64_t)st->cfg.W, lag = (int64_t)st->cfg.lag;
    const int64_t lo = std::max<int64_t>(0, k0 - lag - W);
    std::vector<uint32_t> nz;
    if (known) {
      nz.assign((size_t)(k0 + m - lo + 1), 0);
      for (int64_t q = lo; q < k0 + (int64_t)m; ++q) {
        const uint64_t n = q >= k0 ? h_sizes[first + (uint32_t)(q - k0)] : st->recent[(uint64_t)q % ring];
        nz[(size_t)(q - lo + 1)] = nz[(size_t)(q - lo)] + (n > 0 ? 1u : 0u);
      }
    }
    for (uint32_t j = 0; j < m; ++j) {
      std::memset(&segs[j], 0, sizeof(SegDesc));
      segs[j].ptr = static_cast<const uint8_t *>(h_ptrs[first + j]);
      segs[j].size = h_sizes[first + j];
      segs[j].out = d_out ? d_out + (size_t)(first + j) * 256 : nullptr;
      segs[j].chunk = (int64_t)j;
      segs[j].stream_idx = 0;
      if (known) {
        const int64_t src = k0 + (int64_t)j - 1 - lag;
        if (src < 0) {
          segs[j].known = kKnown | kKnownCold | ((uint32_t)HIST_MODE_WAVEHIST << 16) | ((uint32_t)KIND_UNIFORM << 8);
        } else {
          const int64_t a = std::max<int64_t>(src - W + 1, lo);
          const uint32_t md = nz[(size_t)(src - lo + 1)] > nz[(size_t)(a - lo)] ? HIST_MODE_AHIST : HIST_MODE_WAVEHIST;
          segs[j].known = kKnown | (md << 16) | ((uint32_t)KIND_UNIFORM << 8) | lgmax;
        }
        if (unwalked) {
          // the decision after this chunk, by the same rule: chunks q - W + 1 .. q
          const int64_t q = k0 + (int64_t)j;
          const int64_t a = std::max<int64_t>(q - W + 1, lo);
          if (nz[(size_t)(q - lo + 1)] > nz[(size_t)(a - lo)]) segs[j].known |= kAfterAhist;
          segs[j].known |= kUnwalked;
        }
        if (walk_after) segs[j].known |= kWalkAfter;
      }
    }
    MultiPlan mp;
    // Tiles are handed out in chunk order, so a chunk waiting for an earlier chunk's decision
    // never waits on a workgroup that has not started.  When the host knows every decision
    // nothing waits, and each workgroup takes one equal share of the launch's bytes instead:
    // a share crosses one or two chunk boundaries where dynamic tiles would change chunk at
    // nearly every tile, and equal shares end together where whole tiles would leave some
    // workgroups a tile more than others.
    // When every chunk of the launch takes its decision from an earlier launch (lag + 1 >= m),
    // its chunks wait only on launches that run on their own, never on each other, so equal
    // shares are safe too (with the residency cap of launches that wait, set above).
    const bool ahead = !known && m <= st->cfg.lag + 1;
    const bool split = known || ahead;
    // At lag 0 every chunk waits for the one before it, so the chunks run one at a time: each
    // is cut into one slice per workgroup, and workgroup w counts slice w of every chunk in
    // order (plan_striped).  No tile counter sits on that chain, and a slice is loading while
    // its workgroup waits for the decision.
    bool striped = !split && st->cfg.lag == 0;
    if (striped) {
      const hist_status_t ps = plan_striped(segs, maxg, &mp);
      if (ps == HIST_EOVERFLOW) striped = false;   // slices too large for a tile record
      else TRY(ps);
    }
    if (split) {
      TRY(plan_split(segs, (uint64_t)g_tune[fam].tile_kib * 1024, maxg, &mp));
    } else if (!striped) {
      // Chunks 0 .. m - 2 - lag of this launch make the decisions of its later chunks.  Where
      // those decisions depend on the data, their tiles are cut small (a 64th of a chunk), so
      // that each of them is spread over many workgroups and done soon after its tiles are
      // taken: with whole-grid-sized tiles the first chunks finish only when the grid's first
      // tiles all do, while the tiles of the chunks waiting on them have long been taken and
      // their workgroups spin.  Each small tile costs a flush, though; where every decision is
      // the uniform table (a window stream with the tuned switch) the waits are short anyway
      // and the extra flushes cost more than they save, so those keep the larger tiles.
      const uint32_t producers = (m > st->cfg.lag + 1 && !known) ? m - 1 - st->cfg.lag : 0u;
      uint64_t per_chunk = 0;
      for (uint32_t j = 0; j < m; ++j) per_chunk += h_sizes[first + j];
      per_chunk = std::max<uint64_t>(1, per_chunk / m);
      TRY(plan_multi(segs, tile, maxg, &mp, producers, std::max<uint64_t>(16384, per_chunk / 64)));
    }
    const uint32_t copies = std::min<uint32_t>(64, pow2ceil32(std::max<uint32_t>(1, g_tune[fam].copies)));
    const bool join = known && st->since_join + m > kMaxChunksPerLaunch;
    TRY(stream_launch_begin(st, s, serialize || join));
    st->since_join = join ? m : st->since_join + m;
    TRY(run_multi(d, P, mp, copies, s, nullptr, !split && !striped, true));
    if (walk_after) TRY(dev_err(launch_walk(P, s)));
    stream_launch_end(st, s);
    if (unwalked) st->window_stale = true;
    for (uint32_t j = 0; j < m; ++j) st->recent[(st->pushed + j) % ring] = h_sizes[first + j];
    st->pushed += m;
  }
  return HIST_OK;
}

hist_status_t hist_stream_read(hist_stream_t *st, hist_stream_snapshot_t *snap, uint8_t *h_mode_trace,
                               uint32_t *h_pattern_trace, uint32_t trace_len, void *stream) {
  if (!st) return HIST_EINVAL;
  TRY(stream_sync(st, static_cast<hipStream_t>(stream)));
  if (st->window_stale) {   // nothing of the stream is in flight now
    const hipStream_t s = static_cast<hipStream_t>(stream);
    TRY_HIP(launch_window_rebuild(st->sa.d_st, st->pushed, s));
    TRY_HIP(hipStreamSynchronize(s));
    st->window_stale = false;
  }
  bool timed_out = false;
  if (snap) {
    StreamDev h;
    TRY_HIP(hipMemcpy(&h, st->sa.d_st, sizeof(h), hipMemcpyDeviceToHost));
    std::memset(snap, 0, sizeof(*snap));
    snap->chunks = h.done;
    std::memcpy(snap->acc, h.acc, sizeof(snap->acc));
    std::memcpy(snap->mw, h.mw, sizeof(snap->mw));
    snap->alarms = h.alarms;
    snap->first_alarm = h.first_alarm;
    snap->last_alarm = h.last_alarm;
    snap->wait_timeouts = h.wait_timeouts;
    snap->merge_timeouts = h.merge_timeouts;
    timed_out = h.wait_timeouts != 0 || h.merge_timeouts != 0;
    const bool sequenced = st->cfg.W > 1 || st->cfg.alarm_pct > 0;
    if (h.done > 0) {
      Decision dec;
      TRY_HIP(hipMemcpy(&dec, st->sa.d_slots + (h.done - 1) % st->nslot, sizeof(dec), hipMemcpyDeviceToHost));
      snap->next_mode = tag_mode(dec.tag);
      if (!sequenced)   // the window is the last chunk, kept with its decision
        for (int v = 0; v < 256; ++v) snap->mw[v] = dec.hist[v];
      const uint32_t kl = tag_kind_lg(dec.tag);
      if ((kl >> 8) == KIND_UNIFORM) {   // the words of a uniform pattern are not stored
        const uint32_t lg = kl & 0xFFu;
        for (uint32_t v = 0; v < 256; ++v) snap->next_pattern.word[v] = (v << lg) | (lg << 16);
      } else {
        std::memcpy(snap->next_pattern.word, dec.words, sizeof(dec.words));
      }
      snap->next_pattern.total_S = st->cfg.S;
      snap->next_pattern.rmax = st->cfg.rmax;
    } else {
      snap->next_mode = HIST_MODE_WAVEHIST;
      TRY(hist_pattern_init(&snap->next_pattern, HIST_PAT_IDENTITY, 0, 0));
    }
  }
  const uint32_t n = std::min<uint32_t>(trace_len, st->cfg.trace_cap);
  if (h_mode_trace && n) TRY_HIP(hipMemcpy(h_mode_trace, st->sa.d_mode_trace, n, hipMemcpyDeviceToHost));
  if (h_pattern_trace && n)
    TRY_HIP(hipMemcpy(h_pattern_trace, st->sa.d_pat_trace, (size_t)n * 256 * 4, hipMemcpyDeviceToHost));
  if (!snap) {
    uint64_t to[2];
    TRY_HIP(hipMemcpy(to, &st->sa.d_st->wait_timeouts, sizeof(to), hipMemcpyDeviceToHost));
    timed_out = to[0] != 0 || to[1] != 0;
  }
  return timed_out ? HIST_ETIMEDOUT : HIST_OK;
}

hist_status_t hist_stream_read_alarms(hist_stream_t *st, uint8_t *h_alarm_trace, uint32_t trace_len, void *stream) {
  if (!st || st->cfg.alarm_pct == 0 || (!h_alarm_trace && trace_len > 0)) return HIST_EINVAL;
  TRY(stream_sync(st, static_cast<hipStream_t>(stream)));
  const uint32_t n = std::min<uint32_t>(trace_len, st->cfg.trace_cap);
  if (n)   // the alarm trace follows the mode trace (one stream, trace_cap entries each)
    TRY_HIP(hipMemcpy(h_alarm_trace, st->sa.d_mode_trace + std::max<uint32_t>(st->cfg.trace_cap, 1), n,
                      hipMemcpyDeviceToHost));
  if (trace_len > n) std::memset(h_alarm_trace + n, 0, trace_len - n);
  return HIST_OK;
}

hist_status_t hist_stream_read_times(hist_stream_t *st, uint64_t *h_times_ns, uint32_t trace_len, void *stream) {
  if (!st || (!h_times_ns && trace_len > 0)) return HIST_EINVAL;
  TRY(stream_sync(st, static_cast<hipStream_t>(stream)));
  const uint32_t n = std::min<uint32_t>(trace_len, st->cfg.trace_cap);
  std::vector<uint64_t> raw((size_t)n * 3);
  if (n) TRY_HIP(hipMemcpy(raw.data(), st->sa.d_time_trace, raw.size() * 8, hipMemcpyDeviceToHost));
  int dev = 0, khz = 0;
  TRY_HIP(hipGetDevice(&dev));
  TRY_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) return HIST_EDEVICE;
  for (size_t i = 0; i < raw.size(); ++i) {   // unwritten entries (all ones) -> 0
    const uint64_t x = raw[i];
    if (x == ~0ull) h_times_ns[i] = 0;
    else if (i % 3 == 2) h_times_ns[i] = x;   // MHz as measured
    else h_times_ns[i] = (uint64_t)((long double)x * 1.0e6L / (long double)khz);   // ticks -> ns
  }
  for (size_t i = raw.size(); i < (size_t)trace_len * 3; ++i) h_times_ns[i] = 0;
  return HIST_OK;
}

hist_status_t hist_stream_destroy(hist_stream_t *st) {
  if (!st) return HIST_EINVAL;
  (void)hipDeviceSynchronize();
  stream_state_free(&st->sa);
  for (int i = 0; i < 2; ++i)
    if (st->ev[i]) (void)hipEventDestroy(st->ev[i]);
  delete st;
  return HIST_OK;
}

// ---------------------------------------------------------------- diagnostics and tuning

hist_status_t hist_diag_read(hist_diag_t *out) {
  if (!out) return HIST_EINVAL;
  DevCtx *d;
  TRY(get_dev(&d));
  uint32_t h[64];
  TRY_HIP(hipMemcpy(h, d->diag, sizeof(h), hipMemcpyDeviceToHost));
  uint32_t na[3];
  TRY(noalloc_diag(na));   // launches of hist_u8_noalloc keep their own counters
  out->invalid_patterns = (uint64_t)h[0] + na[0];
  out->wait_timeouts = (uint64_t)h[1] + na[1];
  out->merge_timeouts = (uint64_t)h[2] + na[2];
  return HIST_OK;
}

hist_status_t hist_set_wait_limits(uint32_t decision_polls, uint32_t merge_polls) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_wait_polls = decision_polls ? decision_polls : kDefaultWaitPolls;
  g_merge_polls = merge_polls ? merge_polls : kDefaultMergePolls;
  return HIST_OK;
}

hist_status_t hist_read_probe(const void *d_in, size_t n_bytes, uint64_t *d_sum, uint32_t workgroups,
                              void *stream) {
  if (n_bytes == 0) return HIST_OK;
  if (!d_in || !d_sum || (n_bytes & 15u) || (reinterpret_cast<uintptr_t>(d_in) & 15u) || workgroups > 65536)
    return HIST_EINVAL;
  DevCtx *d;
  TRY(get_dev(&d));
  const uint64_t nvec = (uint64_t)n_bytes >> 4;
  // no more workgroups than the vectors need
  const uint64_t want = std::max<uint64_t>(1, ceil_div(nvec, (uint64_t)kBlock * 4));
  const uint32_t grid = (uint32_t)std::min<uint64_t>(workgroups ? workgroups : (uint64_t)d->cus * 2, want);
  return dev_err(launch_read_probe(d_in, nvec, d_sum, grid, static_cast<hipStream_t>(stream)));
}

hist_status_t hist_tune_set(uint32_t family, const hist_tune_t *t) {
  if (!t || family >= kFamilies) return HIST_EINVAL;
  if (t->tile_kib && (t->tile_kib % 16 || t->tile_kib > (1u << 20))) return HIST_EINVAL;
  if (t->merge_copies && (!is_pow2(t->merge_copies) || t->merge_copies > 64)) return HIST_EINVAL;
  if (t->blocks_per_cu > 8) return HIST_EINVAL;
  if (t->tiles_per_wg > 64) return HIST_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  if (t->blocks_per_cu) g_tune[family].bpc = t->blocks_per_cu;
  if (t->tile_kib) g_tune[family].tile_kib = t->tile_kib;
  if (t->merge_copies) g_tune[family].copies = t->merge_copies;
  if (t->tiles_per_wg) g_tune[family].tpw = t->tiles_per_wg;
  return HIST_OK;
}

hist_status_t hist_tune_get(uint32_t family, hist_tune_t *t) {
  if (!t || family >= kFamilies) return HIST_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  t->blocks_per_cu = g_tune[family].bpc;
  t->tile_kib = g_tune[family].tile_kib;
  t->merge_copies = g_tune[family].copies;
  t->tiles_per_wg = g_tune[family].tpw;
  return HIST_OK;
}

}  // extern "C"
