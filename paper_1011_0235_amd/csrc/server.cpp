// Continuous-batching server of histogram requests (hist_server_*).
//
// Host side: a queue of submitted requests, a scheduler thread, and a pool of micro-batch
// slots (two per HIP stream), each with its own device scratch so slots can run at once.
// The scheduler repeatedly (1) retires finished micro-batches (a lone request's kernel sets a
// word of pinned host memory when its histogram is out; a batch of several completes an
// event, hipEventQuery), freeing their budget and slots, and (2) admits queued requests in arrival order while the budget and the
// slot limit allow, launching each admitted group as one persistent multi-segment kernel.
// Between rounds it spins (no timed sleep: a sleep of a few microseconds is rounded up to
// the kernel's timer slack, tens of microseconds, which would set the latency floor) while
// a batch is in flight and for idle_spin_ns after the last activity; only then does it block
// until a submission wakes it.  Tickets are retired once poll or wait has returned their
// final state, and finished tickets nobody asks about are dropped oldest first beyond
// kFinishedCap, so the host memory a server holds stays bounded.
// Device side: every request is a segment of that launch; its finalizing workgroup writes the
// request's histogram and updates the state of the request's stream id (running uint64
// histogram, moving window of one request, decision) -- see server_epilogue in kernels.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "histmi.h"
#include "histmi_dev.h"
#include "runtime.h"

using namespace histmi;
using namespace histmi::rt;

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Req {
  uint32_t sid = 0;
  const void *buf = nullptr;
  uint64_t n = 0;
  uint32_t *out = nullptr;
  uint64_t t_submit = 0, t_admit = 0, t_done = 0;
  int32_t status = HIST_EBUSY;
};

struct Slot {
  Scratch sc;
  hipEvent_t ev = nullptr;
  // a lone request's launch reports completion through a word of pinned host memory that
  // its finalizer sets to `seq` (no event, no HIP call to notice it); batches of several
  // requests complete `ev`
  volatile uint32_t *done_host = nullptr;
  uint32_t *done_dev = nullptr;
  uint32_t seq = 0;
  bool by_word = false;
  uint64_t t_check = 0;       // last time a wait on the word asked the HIP stream for errors
  // a batch's descriptors, in pinned coherent host memory that its kernel reads in place
  // (rewritten only once the slot's previous launch has finished, since a slot runs one
  // launch at a time): no copy goes through the HIP runtime's copy path, whose first use of
  // a kind can hold the launching thread for milliseconds
  uint8_t *desc_host = nullptr;
  const uint8_t *desc_dev = nullptr;
  size_t desc_cap = 0;
  bool busy = false;
  int hs = 0;
  uint64_t bytes = 0;
  std::vector<uint64_t> tickets;
};

constexpr size_t kQueueCap = 1u << 20;      // not-yet-admitted requests
constexpr size_t kFinishedCap = 1u << 20;   // finished requests kept for poll / wait
constexpr uint64_t kIdleSpinNs = 20000000;  // default of how long the scheduler spins after its last activity
constexpr uint64_t kCheckNs = 100000;
// each slot's scratch is reserved at creation for micro-batches of up to this many requests,
// with descriptor sets of up to kReserveDescBytes (a larger batch grows it on first use)
constexpr uint64_t kReserveSegs = 1024;
constexpr size_t kReserveDescBytes = size_t(4) << 20;       // a launch not done yet: its HIP stream is asked for errors this often

inline void cpu_relax() { __builtin_ia32_pause(); }

}  // namespace

struct hist_server {
  hist_server_config_t cfg;
  int dev = 0;
  DevCtx *d = nullptr;
  StreamAlloc sa;
  std::vector<hipStream_t> hs;
  std::vector<Slot> slots;
  uint32_t *done_words = nullptr;           // pinned host memory: one 64-byte line per slot
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, Req> reqs;   // live tickets: queued, admitted, or finished and not yet retired
  std::deque<uint64_t> finished;            // finished tickets in finishing order (bounds what is kept)
  uint64_t next_ticket = 1;
  std::atomic<uint64_t> submissions{0};     // lets the spinning scheduler notice work without the lock
  std::atomic<bool> stopping{false};
  // longest host calls of the scheduler (written by it alone, read by hist_server_stats)
  std::atomic<uint64_t> max_launch_ns{0}, max_query_ns{0};
  uint64_t idle_spin_ns = kIdleSpinNs;
  uint64_t inflight_bytes = 0, inflight_reqs = 0;
  uint32_t busy_slots = 0;
  bool stop = false;
  hist_server_stats_t stats;
  std::thread th;

  void run();
  bool launch(Slot &sl, std::vector<uint64_t> &batch);
  hipError_t query(Slot &sl);
  hipError_t timed_query(Slot &sl);
  void finish(uint64_t tk, int32_t status, uint64_t t);
};

// Mark an admitted request finished (lock held).
void hist_server::finish(uint64_t tk, int32_t status, uint64_t t) {
  Req &r = reqs[tk];
  r.status = status;
  r.t_done = t;
  inflight_bytes -= r.n;
  inflight_reqs -= 1;
  stats.completed += 1;
  if (status == HIST_OK) stats.bytes_done += r.n;
  finished.push_back(tk);
  while (finished.size() > kFinishedCap) {
    reqs.erase(finished.front());   // no-op if poll or wait already retired it
    finished.pop_front();
  }
}

// Partial copies per segment of a micro-batch of several requests.
static uint32_t multi_copies() {
  return std::min<uint32_t>(64, pow2ceil32(std::max<uint32_t>(1, g_tune[KIND_UNIFORM].copies)));
}

// Launch one micro-batch on slot `sl` (called without the lock; the requests are admitted).
bool hist_server::launch(Slot &sl, std::vector<uint64_t> &batch) {
  Params P;
  init_params(&P);
  stream_layout(cfg.S, cfg.rmax, (hist_mode_t)cfg.mode, &P);
  P.st = sa.d_st;
  std::vector<SegDesc> segs(batch.size());
  {
    std::lock_guard<std::mutex> lk(mu);
    for (size_t j = 0; j < batch.size(); ++j) {
      const Req &r = reqs[batch[j]];
      std::memset(&segs[j], 0, sizeof(SegDesc));
      segs[j].ptr = static_cast<const uint8_t *>(r.buf);
      segs[j].size = r.n;
      segs[j].out = r.out;
      segs[j].chunk = kServerChunk;
      segs[j].stream_idx = r.sid;
    }
  }
  hipStream_t s = hs[sl.hs];
  if (segs.size() == 1) {
    // a lone request spreads over the whole grid with no descriptors to upload (the
    // launch carries it), so nothing but the kernel is queued; sl.ev completes with it
    P.seg0 = segs[0];
    P.done_seq = ++sl.seq;
    P.host_done = sl.done_dev;
    sl.by_word = true;
    sl.t_check = now_ns();
    return run_single(d, P, s, &sl.sc) == HIST_OK;
  }
  sl.by_word = false;
  const uint32_t fam = KIND_UNIFORM;
  const uint64_t tile = (uint64_t)g_tune[fam].tile_kib * 1024;
  const uint32_t maxg = (uint32_t)d->cus * blocks_per_cu(fam, lds_bytes(P));
  MultiPlan mp;
  if (plan_split(segs, tile, maxg, &mp) != HIST_OK) return false;
  const uint32_t copies = multi_copies();
  // sl.ev completes with the launch (the slot's scratch only ever serves this HIP stream);
  // descriptors beyond the slot's host buffer (a batch larger than reserved) are uploaded
  const uint8_t *in_place = nullptr;
  if (mp.blob.size() <= sl.desc_cap) {
    std::memcpy(sl.desc_host, mp.blob.data(), mp.blob.size());
    in_place = sl.desc_dev;
  }
  return run_multi(d, P, mp, copies, s, &sl.sc, false, true, sl.ev, in_place) == HIST_OK;
}

// State of the slot's launch: hipSuccess once done, hipErrorNotReady while it runs, or the
// HIP error that ended it.  A launch that reports through the host word is done when the
// word holds its sequence number; while it is not, the HIP stream is asked now and then, so
// a launch that failed on the device is noticed too (its stream reports the error; a stream
// with nothing left to run and the word still short would be a lost report).
hipError_t hist_server::query(Slot &sl) {
  if (!sl.by_word) return hipEventQuery(sl.ev);
  if (*sl.done_host == sl.seq) return hipSuccess;
  const uint64_t t = now_ns();
  if (t - sl.t_check < kCheckNs) return hipErrorNotReady;
  sl.t_check = t;
  const hipError_t e = hipStreamQuery(hs[sl.hs]);
  if (e == hipErrorNotReady) return e;
  if (*sl.done_host == sl.seq) return hipSuccess;   // the launch ended after writing the word
  return e == hipSuccess ? hipErrorUnknown : e;
}

// query() with its duration kept in max_query_ns (scheduler thread only).
hipError_t hist_server::timed_query(Slot &sl) {
  const uint64_t t0 = now_ns();
  const hipError_t e = query(sl);
  const uint64_t dt = now_ns() - t0;
  if (dt > max_query_ns.load(std::memory_order_relaxed)) max_query_ns.store(dt, std::memory_order_relaxed);
  return e;
}

void hist_server::run() {
  (void)hipSetDevice(dev);
  std::unique_lock<std::mutex> lk(mu);
  uint64_t last_active = now_ns();
  for (;;) {
    // 1. retire finished micro-batches
    for (Slot &sl : slots) {
      if (!sl.busy) continue;
      const hipError_t e = timed_query(sl);
      if (e == hipErrorNotReady) continue;
      const uint64_t t = now_ns();
      for (uint64_t tk : sl.tickets) finish(tk, e == hipSuccess ? HIST_OK : HIST_EDEVICE, t);
      sl.tickets.clear();
      sl.busy = false;
      busy_slots -= 1;
      last_active = t;
      cv_done.notify_all();
    }
    // 2. admit queued requests into free slots
    for (Slot &sl : slots) {
      if (sl.busy || pending.empty()) continue;
      std::vector<uint64_t> batch;
      uint64_t bytes = 0;
      const uint64_t t = now_ns();
      while (!pending.empty() && batch.size() < cfg.max_batch) {
        Req &r = reqs[pending.front()];
        if (inflight_bytes + r.n > cfg.hbm_budget_bytes || inflight_reqs + 1 > cfg.max_slots) break;
        batch.push_back(pending.front());
        pending.pop_front();
        inflight_bytes += r.n;
        inflight_reqs += 1;
        bytes += r.n;
        r.t_admit = t;
      }
      if (batch.empty()) break;
      stats.max_inflight_bytes = std::max(stats.max_inflight_bytes, inflight_bytes);
      stats.max_inflight_requests = std::max(stats.max_inflight_requests, inflight_reqs);
      sl.busy = true;
      busy_slots += 1;
      sl.bytes = bytes;
      stats.batches += 1;
      stats.max_concurrent_batches = std::max<uint64_t>(stats.max_concurrent_batches, busy_slots);
      last_active = t;
      lk.unlock();
      const uint64_t tl = now_ns();
      const bool ok = launch(sl, batch);
      const uint64_t dl = now_ns() - tl;
      if (dl > max_launch_ns.load(std::memory_order_relaxed)) max_launch_ns.store(dl, std::memory_order_relaxed);
      lk.lock();
      sl.tickets = batch;
      if (!ok) {
        // the launch never reached the device: fail these requests now
        const uint64_t tf = now_ns();
        for (uint64_t tk : batch) finish(tk, HIST_EDEVICE, tf);
        sl.tickets.clear();
        sl.busy = false;
        busy_slots -= 1;
        cv_done.notify_all();
      }
    }
    if (stop && pending.empty() && busy_slots == 0) break;
    // 3. wait for work: spin while a batch is in flight or work came recently, else block.
    // (Whatever is still pending now waits for a batch to finish: every free slot was
    // offered the queue's front.)  Only this thread changes the slots, so they are read
    // here without the lock.
    const uint64_t seen = submissions.load(std::memory_order_acquire);
    const bool inflight = busy_slots > 0;
    if (!inflight && pending.empty() && now_ns() - last_active > idle_spin_ns) {
      if (stop) break;
      cv_work.wait(lk, [this] { return stop || !pending.empty(); });
      last_active = now_ns();
      continue;
    }
    lk.unlock();
    for (uint32_t spins = 0;; ++spins) {
      bool done = false;
      for (Slot &sl : slots)
        if (sl.busy && timed_query(sl) != hipErrorNotReady) {
          done = true;
          break;
        }
      if (done || submissions.load(std::memory_order_acquire) != seen || (stopping.load() && !inflight)) break;
      if (!inflight && now_ns() - last_active > idle_spin_ns) break;
      for (int i = 0; i < 32; ++i) cpu_relax();
    }
    lk.lock();
  }
}

extern "C" {

hist_status_t hist_server_destroy(hist_server_t *sv);

hist_status_t hist_server_create(hist_server_t **out, const hist_server_config_t *cfg) {
  if (!out || !cfg) return HIST_EINVAL;
  const hist_server_config_t c = *cfg;
  if (c.hbm_budget_bytes == 0 || c.max_slots < 1 || c.n_stream_ids < 1 || c.n_stream_ids > 65536 ||
      c.n_hip_streams < 1 || c.n_hip_streams > 16 || c.max_batch < 1 || c.max_batch > 65536 ||
      !mode_ok((hist_mode_t)c.mode) || c.theta_pct > 100 || c.S < 256 || c.S > HIST_S_MAX || !is_pow2(c.rmax) ||
      c.rmax > HIST_RMAX_MAX || c.idle_spin_us > 10000000u)
    return HIST_EINVAL;
  DevCtx *d;
  TRY(get_dev(&d));
  hist_server *sv = new hist_server();
  sv->cfg = c;
  if (c.idle_spin_us) sv->idle_spin_ns = (uint64_t)c.idle_spin_us * 1000u;
  sv->dev = d->dev;
  sv->d = d;
  std::memset(&sv->stats, 0, sizeof(sv->stats));
  hist_status_t st = stream_state_alloc(c.n_stream_ids, 1, c.theta_pct, c.S, c.rmax, 0, 1, 0, 0, &sv->sa);
  if (st != HIST_OK) {
    delete sv;
    return st;
  }
  sv->hs.resize(c.n_hip_streams, nullptr);
  for (auto &h : sv->hs) {
    if (hipStreamCreateWithFlags(&h, hipStreamNonBlocking) != hipSuccess) {
      hist_server_destroy(sv);
      return HIST_EDEVICE;
    }
  }
  sv->slots.resize((size_t)c.n_hip_streams * 2);
  if (hipHostMalloc(reinterpret_cast<void **>(&sv->done_words), sv->slots.size() * 64, hipHostMallocCoherent) !=
      hipSuccess) {
    sv->done_words = nullptr;
    hist_server_destroy(sv);
    return HIST_ENOMEM;
  }
  std::memset(sv->done_words, 0, sv->slots.size() * 64);
  for (size_t i = 0; i < sv->slots.size(); ++i) {
    sv->slots[i].hs = (int)(i % c.n_hip_streams);
    sv->slots[i].done_host = sv->done_words + i * 16;
    void *dp = nullptr;
    if (hipHostGetDevicePointer(&dp, sv->done_words + i * 16, 0) != hipSuccess) {
      hist_server_destroy(sv);
      return HIST_EDEVICE;
    }
    sv->slots[i].done_dev = static_cast<uint32_t *>(dp);
    if (hipEventCreateWithFlags(&sv->slots[i].ev, hipEventDisableTiming) != hipSuccess) {
      hist_server_destroy(sv);
      return HIST_EDEVICE;
    }
  }
  // Reserve every slot's scratch for the largest micro-batch the server launches, and a host
  // buffer for its largest descriptor set, so that the scheduler's launches allocate and copy
  // nothing: a buffer grown in the launch path costs a hipFree and a hipMalloc, which wait
  // for the whole device and held up every slot's completion and admission for milliseconds.
  {
    Params P;
    init_params(&P);
    stream_layout(c.S, c.rmax, (hist_mode_t)c.mode, &P);
    const uint32_t maxg = (uint32_t)d->cus * blocks_per_cu(KIND_UNIFORM, lds_bytes(P));
    const uint64_t nseg = std::min<uint64_t>({(uint64_t)c.max_batch, (uint64_t)c.max_slots, kReserveSegs});
    const uint32_t copies = std::max<uint32_t>(g_single_copies, multi_copies());
    const uint64_t bytes = std::min<uint64_t>(c.hbm_budget_bytes, nseg * kMaxSegBytes);
    const size_t desc = std::max<size_t>(
        4096, std::min<size_t>(plan_split_blob_max(nseg, bytes, (uint64_t)g_tune[KIND_UNIFORM].tile_kib * 1024, maxg),
                               kReserveDescBytes));
    for (Slot &sl : sv->slots) {
      const hist_status_t rs = reserve_scratch(&sl.sc, nseg, copies, 0, sv->hs[sl.hs]);
      if (rs != HIST_OK) {
        hist_server_destroy(sv);
        return rs;
      }
      void *hp = nullptr, *dp = nullptr;
      if (hipHostMalloc(&hp, desc, hipHostMallocCoherent) != hipSuccess) {
        hist_server_destroy(sv);
        return HIST_ENOMEM;
      }
      sl.desc_host = static_cast<uint8_t *>(hp);
      if (hipHostGetDevicePointer(&dp, hp, 0) != hipSuccess) {
        hist_server_destroy(sv);
        return HIST_EDEVICE;
      }
      sl.desc_dev = static_cast<const uint8_t *>(dp);
      sl.desc_cap = desc;
    }
    for (hipStream_t h : sv->hs)
      if (hipStreamSynchronize(h) != hipSuccess) {
        hist_server_destroy(sv);
        return HIST_EDEVICE;
      }
  }
  // every ticket the server can hold at once (queued, in flight, finished and not yet
  // retired) fits without a rehash, which would hold the lock for milliseconds at 10^5 entries
  sv->reqs.reserve(kQueueCap + kFinishedCap + c.max_slots + 1);
  sv->th = std::thread([sv] { sv->run(); });
  *out = sv;
  return HIST_OK;
}

hist_status_t hist_server_submit(hist_server_t *sv, uint32_t stream_id, const void *d_buf, size_t n, uint32_t *d_out,
                                 uint64_t *ticket) {
  if (!sv || !ticket || stream_id >= sv->cfg.n_stream_ids || (n && !d_buf)) return HIST_EINVAL;
  if ((uint64_t)n > kMaxSegBytes) return HIST_EOVERFLOW;
  if ((uint64_t)n > sv->cfg.hbm_budget_bytes) return HIST_EINVAL;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return HIST_ECANCELED;
    if (sv->pending.size() >= kQueueCap) return HIST_EBUSY;
    const uint64_t tk = sv->next_ticket++;
    Req &r = sv->reqs[tk];
    r.sid = stream_id;
    r.buf = d_buf;
    r.n = n;
    r.out = d_out;
    r.t_submit = now_ns();
    *ticket = tk;
    sv->pending.push_back(tk);
    sv->stats.submitted += 1;
    sv->submissions.fetch_add(1, std::memory_order_release);
  }
  sv->cv_work.notify_one();
  return HIST_OK;
}

static void fill_result(const Req &r, hist_server_result_t *out) {
  out->status = r.status;
  out->stream_id = r.sid;
  out->bytes = r.n;
  out->t_submit_ns = r.t_submit;
  out->t_admit_ns = r.t_admit;
  out->t_done_ns = r.t_done;
}

// Fill r from a live ticket; a finished one is retired (lock held).
static void report(hist_server *sv, std::unordered_map<uint64_t, Req>::iterator it, hist_server_result_t *r) {
  if (r) fill_result(it->second, r);
  if (it->second.status != HIST_EBUSY) sv->reqs.erase(it);
}

hist_status_t hist_server_poll(hist_server_t *sv, uint64_t ticket, hist_server_result_t *r) {
  if (!sv || !r) return HIST_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return HIST_EINVAL;
  report(sv, it, r);
  return HIST_OK;
}

hist_status_t hist_server_wait(hist_server_t *sv, uint64_t ticket, int64_t timeout_ns, hist_server_result_t *r) {
  if (!sv) return HIST_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->reqs.find(ticket) == sv->reqs.end()) return HIST_EINVAL;
  // the ticket stays live until this call retires it (only poll or wait retire a ticket, and
  // one ticket is waited on by one thread); finished tickets are not dropped for the cap
  // while this thread waits for the lock, since that only happens after 2^20 later ones
  auto done = [&] {
    auto it = sv->reqs.find(ticket);
    return it == sv->reqs.end() || it->second.status != HIST_EBUSY;
  };
  bool ok = true;
  if (timeout_ns < 0) sv->cv_done.wait(lk, done);
  else ok = sv->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), done);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return HIST_EINVAL;
  report(sv, it, r);
  return ok ? HIST_OK : HIST_ETIMEDOUT;
}

hist_status_t hist_server_drain(hist_server_t *sv, int64_t timeout_ns) {
  if (!sv) return HIST_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto idle = [&] { return sv->pending.empty() && sv->busy_slots == 0; };
  if (timeout_ns < 0) {
    sv->cv_done.wait(lk, idle);
    return HIST_OK;
  }
  return sv->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), idle) ? HIST_OK : HIST_ETIMEDOUT;
}

hist_status_t hist_server_stream_acc(hist_server_t *sv, uint32_t stream_id, uint64_t *h_acc) {
  if (!sv || !h_acc || stream_id >= sv->cfg.n_stream_ids) return HIST_EINVAL;
  const StreamDev *p = sv->sa.d_st + stream_id;
  TRY_HIP(hipMemcpy(h_acc, &p->acc[0], 256 * sizeof(uint64_t), hipMemcpyDeviceToHost));
  return HIST_OK;
}

hist_status_t hist_server_stats(hist_server_t *sv, hist_server_stats_t *st) {
  if (!sv || !st) return HIST_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  *st = sv->stats;
  st->max_launch_ns = sv->max_launch_ns.load(std::memory_order_relaxed);
  st->max_query_ns = sv->max_query_ns.load(std::memory_order_relaxed);
  return HIST_OK;
}

hist_status_t hist_server_destroy(hist_server_t *sv) {
  if (!sv) return HIST_EINVAL;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->stopping.store(true);
    for (uint64_t tk : sv->pending) {
      Req &r = sv->reqs[tk];
      r.status = HIST_ECANCELED;
      r.t_done = now_ns();
      sv->stats.canceled += 1;
    }
    sv->pending.clear();
  }
  sv->cv_work.notify_all();
  sv->cv_done.notify_all();
  if (sv->th.joinable()) sv->th.join();   // the thread exits once every admitted batch retired
  // a launch that reported through its host word may still be ending: let every HIP stream
  // drain before its scratch and the words are freed
  for (hipStream_t h : sv->hs)
    if (h) (void)hipStreamSynchronize(h);
  for (Slot &sl : sv->slots) {
    free_scratch(&sl.sc);
    if (sl.desc_host) (void)hipHostFree(sl.desc_host);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
  }
  for (hipStream_t h : sv->hs)
    if (h) (void)hipStreamDestroy(h);
  if (sv->done_words) (void)hipHostFree(sv->done_words);
  stream_state_free(&sv->sa);
  delete sv;
  return HIST_OK;
}

}  // extern "C"
