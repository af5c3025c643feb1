// Host-ingest streams (hist_ingest_*): chunks in host memory are copied to the device and
// pushed through a device-resident stream, the copies overlapping the counting across a set
// of HIP streams used in turn (the paper's pipelined stream, Sec. III.B).
//
// Each HIP stream owns one device staging buffer.  A push queues, on the next HIP stream,
// the host-to-device copy into that stream's buffer and then the chunk's launch; the next
// copy into the same buffer is queued on the same HIP stream, so it waits for that launch.
// Different HIP streams run their copies and launches independently, and the stream object
// makes each chunk wait on the device for the decision it runs with.

#include <hip/hip_runtime.h>

#include <vector>

#include "histmi.h"
#include "histmi_dev.h"
#include "runtime.h"

using namespace histmi;
using namespace histmi::rt;

struct hist_ingest {
  hist_ingest_config_t cfg{};
  std::vector<hipStream_t> hs;
  std::vector<void *> staging;
  uint32_t next = 0;
};

namespace {

void ingest_free(hist_ingest *ing) {
  for (hipStream_t s : ing->hs)
    if (s) (void)hipStreamSynchronize(s);
  for (void *p : ing->staging)
    if (p) (void)hipFree(p);
  for (hipStream_t s : ing->hs)
    if (s) (void)hipStreamDestroy(s);
  delete ing;
}

}  // namespace

extern "C" {

hist_status_t hist_ingest_create(hist_ingest_t **out, const hist_ingest_config_t *cfg) {
  if (!out || !cfg) return HIST_EINVAL;
  if (cfg->n_hip_streams < 1 || cfg->n_hip_streams > 256 || cfg->slot_bytes == 0 || cfg->slot_bytes > kMaxSegBytes)
    return HIST_EINVAL;
  DevCtx *d;
  TRY(get_dev(&d));
  hist_ingest *ing = new hist_ingest();
  ing->cfg = *cfg;
  ing->hs.assign(cfg->n_hip_streams, nullptr);
  ing->staging.assign(cfg->n_hip_streams, nullptr);
  for (uint32_t j = 0; j < cfg->n_hip_streams; ++j) {
    if (hipStreamCreateWithFlags(&ing->hs[j], hipStreamNonBlocking) != hipSuccess) {
      ing->hs[j] = nullptr;
      ingest_free(ing);
      return HIST_EDEVICE;
    }
    if (hipMalloc(&ing->staging[j], (size_t)cfg->slot_bytes) != hipSuccess) {
      ing->staging[j] = nullptr;
      ingest_free(ing);
      return HIST_ENOMEM;
    }
  }
  *out = ing;
  return HIST_OK;
}

hist_status_t hist_ingest_push(hist_ingest_t *ing, hist_stream_t *st, const void *h_chunk, size_t n,
                               hist_mode_t mode, uint32_t *d_out_k) {
  if (!ing || !st || (n && !h_chunk) || (uint64_t)n > ing->cfg.slot_bytes || !mode_ok(mode)) return HIST_EINVAL;
  const uint32_t j = ing->next;
  hipStream_t s = ing->hs[j];
  if (n) TRY_HIP(hipMemcpyAsync(ing->staging[j], h_chunk, n, hipMemcpyHostToDevice, s));
  TRY(hist_stream_push(st, n ? ing->staging[j] : nullptr, n, mode, d_out_k, s));
  ing->next = (j + 1) % ing->cfg.n_hip_streams;
  return HIST_OK;
}

hist_status_t hist_ingest_sync(hist_ingest_t *ing) {
  if (!ing) return HIST_EINVAL;
  for (hipStream_t s : ing->hs) TRY_HIP(hipStreamSynchronize(s));
  return HIST_OK;
}

hist_status_t hist_ingest_destroy(hist_ingest_t *ing) {
  if (!ing) return HIST_EINVAL;
  ingest_free(ing);
  return HIST_OK;
}

}  // extern "C"
