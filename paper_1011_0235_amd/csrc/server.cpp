// Continuous-batching server of histogram requests (hist_server_*).
//
// Host side: a queue of submitted requests, a scheduler thread, and a pool of micro-batch
// slots (two per HIP stream), each with its own device scratch so slots can run at once.
// The scheduler repeatedly (1) retires finished micro-batches (hipEventQuery), freeing their
// budget and slots, and (2) admits queued requests in arrival order while the budget and the
// slot limit allow, launching each admitted group as one persistent multi-segment kernel.
// Device side: every request is a segment of that launch; its finalizing workgroup writes the
// request's histogram and updates the state of the request's stream id (running uint64
// histogram, moving window of one request, decision) -- see server_epilogue in kernels.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
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
  bool busy = false;
  int hs = 0;
  uint64_t bytes = 0;
  std::vector<uint64_t> tickets;
};

constexpr size_t kQueueCap = 1u << 20;   // not-yet-admitted requests

}  // namespace

struct hist_server {
  hist_server_config_t cfg;
  int dev = 0;
  DevCtx *d = nullptr;
  StreamAlloc sa;
  std::vector<hipStream_t> hs;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> pending;
  std::vector<Req> reqs;            // ticket t lives at reqs[t - 1]
  uint64_t inflight_bytes = 0, inflight_reqs = 0;
  uint32_t busy_slots = 0;
  bool stop = false;
  hist_server_stats_t stats;
  std::thread th;

  void run();
  bool launch(Slot &sl, std::vector<uint64_t> &batch);
};

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
      const Req &r = reqs[batch[j] - 1];
      std::memset(&segs[j], 0, sizeof(SegDesc));
      segs[j].ptr = static_cast<const uint8_t *>(r.buf);
      segs[j].size = r.n;
      segs[j].out = r.out;
      segs[j].chunk = kServerChunk;
      segs[j].stream_idx = r.sid;
    }
  }
  const uint32_t fam = KIND_UNIFORM;
  const uint64_t tile = (uint64_t)g_tune[fam].tile_kib * 1024;
  const uint32_t maxg = (uint32_t)d->cus * blocks_per_cu(fam, lds_bytes(P));
  MultiPlan mp;
  if (plan_split(segs, tile, maxg, &mp) != HIST_OK) return false;
  const uint32_t copies = std::min<uint32_t>(64, pow2ceil32(std::max<uint32_t>(1, g_tune[fam].copies)));
  hipStream_t s = hs[sl.hs];
  if (run_multi(d, P, mp, copies, s, &sl.sc, false, true) != HIST_OK) return false;
  return hipEventRecord(sl.ev, s) == hipSuccess;
}

void hist_server::run() {
  (void)hipSetDevice(dev);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // 1. retire finished micro-batches
    for (Slot &sl : slots) {
      if (!sl.busy) continue;
      const hipError_t e = hipEventQuery(sl.ev);
      if (e == hipErrorNotReady) continue;
      const uint64_t t = now_ns();
      for (uint64_t tk : sl.tickets) {
        Req &r = reqs[tk - 1];
        r.status = (e == hipSuccess) ? HIST_OK : HIST_EDEVICE;
        r.t_done = t;
        inflight_bytes -= r.n;
        inflight_reqs -= 1;
        stats.completed += 1;
        if (e == hipSuccess) stats.bytes_done += r.n;
      }
      sl.tickets.clear();
      sl.busy = false;
      busy_slots -= 1;
      cv_done.notify_all();
    }
    // 2. admit queued requests into free slots
    for (Slot &sl : slots) {
      if (sl.busy || pending.empty()) continue;
      std::vector<uint64_t> batch;
      uint64_t bytes = 0;
      const uint64_t t = now_ns();
      while (!pending.empty() && batch.size() < cfg.max_batch) {
        Req &r = reqs[pending.front() - 1];
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
      lk.unlock();
      const bool ok = launch(sl, batch);
      lk.lock();
      sl.tickets = batch;
      if (!ok) {
        // the launch never reached the device: fail these requests now
        for (uint64_t tk : batch) {
          Req &r = reqs[tk - 1];
          r.status = HIST_EDEVICE;
          r.t_done = now_ns();
          inflight_bytes -= r.n;
          inflight_reqs -= 1;
          stats.completed += 1;
        }
        sl.tickets.clear();
        sl.busy = false;
        busy_slots -= 1;
        cv_done.notify_all();
      }
    }
    // 3. wait for work
    if (busy_slots > 0) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(2));
      lk.lock();
    } else if (pending.empty()) {
      if (stop) break;
      cv_work.wait(lk, [this] { return stop || !pending.empty(); });
      if (stop && pending.empty()) break;
    }
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
      c.rmax > HIST_RMAX_MAX)
    return HIST_EINVAL;
  DevCtx *d;
  TRY(get_dev(&d));
  hist_server *sv = new hist_server();
  sv->cfg = c;
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
  for (size_t i = 0; i < sv->slots.size(); ++i) {
    sv->slots[i].hs = (int)(i % c.n_hip_streams);
    if (hipEventCreateWithFlags(&sv->slots[i].ev, hipEventDisableTiming) != hipSuccess) {
      hist_server_destroy(sv);
      return HIST_EDEVICE;
    }
  }
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
    Req r;
    r.sid = stream_id;
    r.buf = d_buf;
    r.n = n;
    r.out = d_out;
    r.t_submit = now_ns();
    sv->reqs.push_back(r);
    *ticket = sv->reqs.size();
    sv->pending.push_back(*ticket);
    sv->stats.submitted += 1;
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

hist_status_t hist_server_poll(hist_server_t *sv, uint64_t ticket, hist_server_result_t *r) {
  if (!sv || !r) return HIST_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (ticket == 0 || ticket > sv->reqs.size()) return HIST_EINVAL;
  fill_result(sv->reqs[ticket - 1], r);
  return HIST_OK;
}

hist_status_t hist_server_wait(hist_server_t *sv, uint64_t ticket, int64_t timeout_ns, hist_server_result_t *r) {
  if (!sv) return HIST_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  if (ticket == 0 || ticket > sv->reqs.size()) return HIST_EINVAL;
  auto done = [&] { return sv->reqs[ticket - 1].status != HIST_EBUSY; };
  if (timeout_ns < 0) {
    sv->cv_done.wait(lk, done);
  } else if (!sv->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), done)) {
    if (r) fill_result(sv->reqs[ticket - 1], r);
    return HIST_ETIMEDOUT;
  }
  if (r) fill_result(sv->reqs[ticket - 1], r);
  return HIST_OK;
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
  return HIST_OK;
}

hist_status_t hist_server_destroy(hist_server_t *sv) {
  if (!sv) return HIST_EINVAL;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    for (uint64_t tk : sv->pending) {
      Req &r = sv->reqs[tk - 1];
      r.status = HIST_ECANCELED;
      r.t_done = now_ns();
      sv->stats.canceled += 1;
    }
    sv->pending.clear();
  }
  sv->cv_work.notify_all();
  sv->cv_done.notify_all();
  if (sv->th.joinable()) sv->th.join();   // the thread exits once every admitted batch retired
  for (Slot &sl : sv->slots) {
    free_scratch(&sl.sc);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
  }
  for (hipStream_t h : sv->hs)
    if (h) (void)hipStreamDestroy(h);
  stream_state_free(&sv->sa);
  delete sv;
  return HIST_OK;
}

}  // extern "C"
