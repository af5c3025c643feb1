// Internal host runtime of libhistmi (shared by the C ABI and the server).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "histmi.h"
#include "histmi_dev.h"

namespace histmi {

// kernels.hip
// `done`, if not null, completes when the kernel does (recorded by the dispatch itself).
hipError_t launch_hist(const Params &P, const LaunchShape &sh, hipStream_t s, hipEvent_t done = nullptr);
hipError_t launch_pattern_update(const uint64_t *h, uint32_t S, uint32_t rmax, hist_pattern_t *out, hipStream_t s);
hipError_t launch_read_probe(const void *d_in, uint64_t nvec, uint64_t *d_sum, uint32_t grid, hipStream_t s);
// the in-order walk of a stream launch's chunks (kWalkAfter), after that launch on `s`
hipError_t launch_walk(const Params &P, hipStream_t s);
// a window stream's window (MW, its bytes, the walk's position) rebuilt from its ring at chunk n
hipError_t launch_window_rebuild(StreamDev *st, uint64_t n, hipStream_t s);
hipError_t set_kernel_attrs(uint32_t max_dyn_lds);
hipError_t occupancy(uint32_t lds_bytes, int *blocks_per_cu);
uint32_t ctl_bytes();   // control block at the end of the dynamic LDS
// noalloc.hip: diagnostics counters of hist_u8_noalloc launches on the current device
hist_status_t noalloc_diag(uint32_t out[3]);

namespace rt {

constexpr uint32_t kStaticLdsReserve = 8192;       // static LDS of the kernel (control block), with margin
constexpr uint64_t kMaxSegBytes = 0xFFFFFFFFull;   // per-segment counts must fit the 32-bit partials
constexpr uint32_t kFamilies = 6;                  // one tuning entry per Kind, then ordered streams
constexpr uint32_t kFamStream = HIST_TUNE_STREAM;
constexpr uint32_t kFamStreamKnown = HIST_TUNE_STREAM_KNOWN;
constexpr uint32_t kMaxChunksPerLaunch = 1024;     // stream chunks in one persistent launch, at most

#define TRY_HIP(x)                               \
  do {                                           \
    hipError_t e_ = (x);                         \
    if (e_ != hipSuccess) return HIST_EDEVICE;   \
  } while (0)
#define TRY(x)                        \
  do {                                \
    hist_status_t s_ = (x);           \
    if (s_ != HIST_OK) return s_;     \
  } while (0)

inline hist_status_t dev_err(hipError_t e) { return e == hipSuccess ? HIST_OK : HIST_EDEVICE; }
inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline uint32_t pow2ceil32(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}
inline uint32_t log2u(uint32_t x) {
  uint32_t l = 0;
  while ((1u << l) < x) ++l;
  return l;
}
inline bool is_pow2(uint32_t x) { return x && !(x & (x - 1)); }
inline bool mode_ok(hist_mode_t m) {
  return m == HIST_MODE_AUTO || m == HIST_MODE_AHIST || m == HIST_MODE_WAVEHIST || m == HIST_MODE_WAVEAGG;
}

struct Tune {
  uint32_t bpc;        // workgroups per CU
  uint32_t tile_kib;   // largest multi-segment tile
  uint32_t copies;     // partial copies per segment (multi-segment launches)
  uint32_t tpw;        // multi-segment launches: about this many tiles per workgroup
};
extern Tune g_tune[kFamilies];
extern uint32_t g_single_copies;

// Library-owned device scratch of one launch context (a HIP stream, a graph or a server slot).
// ctr, seg_done and partial are all-zero between launches: each launch's finalizers reset them.
struct Scratch {
  uint32_t *ctr = nullptr;        // 64 words
  size_t ctr_cap = 0;
  uint32_t *seg_done = nullptr;
  size_t seg_cap = 0;
  uint32_t *partial = nullptr;    // words
  size_t partial_cap = 0;
  uint8_t *desc = nullptr;        // device descriptors the next launch reads (segments, tile map, bounds)
  uint8_t *desc_buf = nullptr;    // dedicated descriptor buffer (graphs), owned
  size_t desc_cap = 0;
  uint8_t *stage[2] = {nullptr, nullptr};   // pinned host staging of descriptors
  size_t stage_cap[2] = {0, 0};
  hipEvent_t ev[2] = {nullptr, nullptr};
  int turn = 0;
  // recently uploaded descriptor sets, each in its own device buffer (an identical set is
  // reused without a copy); `desc` points at the one the next launch uses.  A Scratch serves
  // launches on one HIP stream only, so a refill (a copy on that stream) never overtakes a
  // launch still reading the entry.
  struct Cached {
    std::vector<uint8_t> blob;
    uint8_t *dev = nullptr;
    size_t cap = 0;
    uint64_t used = 0;
  };
  Cached cache[4];
  int cur = -1;                   // cache entry `desc` points at (-1: desc_buf)
  uint64_t tick = 0;
};
void free_scratch(Scratch *sc);

struct DevCtx {
  int dev = 0;
  int cus = 0;
  size_t lds_cu = 0;
  uint32_t *diag = nullptr;   // device counters (64 words)
  std::unordered_map<hipStream_t, Scratch *> scratch;
};

hist_status_t get_dev(DevCtx **out);
hist_status_t alloc_scratch(Scratch *sc, size_t nseg, uint32_t copies, size_t desc_bytes, hipStream_t s);
hist_status_t get_scratch(DevCtx *d, hipStream_t s, size_t nseg, uint32_t copies, size_t desc_bytes, Scratch **out);
hist_status_t upload_desc(Scratch *sc, const void *host, size_t bytes, hipStream_t s);
// Allocate now everything that launches of up to nseg segments with up to `copies` partial
// copies, and descriptor sets of up to desc_bytes uploaded through upload_desc, will use, so
// that those launches make no allocation (whose device-wide waits would stall the caller).
hist_status_t reserve_scratch(Scratch *sc, size_t nseg, uint32_t copies, size_t desc_bytes, hipStream_t s);

bool pattern_ok(const hist_pattern_t *p);
void init_params(Params *P);
// Kind and LDS layout of a history-free launch.
hist_status_t select_kind(hist_mode_t mode, const hist_pattern_t *h_pat, Params *P);
// Kind capacity and LDS layout of a launch whose chunks follow device-resident decisions.
void stream_layout(uint32_t S, uint32_t rmax, hist_mode_t mode, Params *P);
uint32_t lds_bytes(const Params &P);
uint32_t resident_per_cu(uint32_t lds);
uint32_t blocks_per_cu(uint32_t family, uint32_t lds);

// One segment cut into one tile per workgroup.  own: a scratch that only launches on `s`
// use, or nullptr for the HIP stream's own; done: as for launch_hist.
hist_status_t run_single(DevCtx *d, Params &P, hipStream_t s, Scratch *own = nullptr, hipEvent_t done = nullptr);

// Segments + tile map + per-workgroup bounds in one host buffer.
struct MultiPlan {
  std::vector<uint8_t> blob;   // SegDesc[n] | TileRec[ntiles] | uint32 bounds[grid + 1] | WgStart[grid] (static)
  uint32_t nseg = 0;
  uint32_t ntiles = 0;
  uint32_t grid = 0;
  size_t seg_bytes = 0;
  size_t rec_bytes = 0;
  size_t start_off = 0;        // offset of the WgStart section (static plans), 0 if none
};
// segs: ptr/size/out/acc/chunk/stream_idx filled; tile0/ntiles are filled here.
// Launches whose chunks may wait: tiles of at most `tile` bytes, in segment order, handed out
// by the launch's counter.
// Tiles in segment order for a launch that hands them out dynamically; the first n_small
// segments are cut into tiles of at most small_tile bytes (0: all tiles up to `tile`).
hist_status_t plan_multi(std::vector<SegDesc> &segs, uint64_t tile, uint32_t max_grid, MultiPlan *mp,
                         uint32_t n_small = 0, uint64_t small_tile = 0);
// Static launches that never wait: one equal share of the launch's bytes per workgroup,
// cut at 16 KiB steps from each segment's start into tiles of at most `tile` bytes.  Each
// segment also costs its workgroups a switch (flush, merge, next descriptor), about what
// one workgroup counts in 4-5 us, so a segment's start is charged 64 KiB on the axis the
// shares are cut from.
hist_status_t plan_split(std::vector<SegDesc> &segs, uint64_t tile, uint32_t max_grid, MultiPlan *mp);
// An upper bound on plan_split's descriptor bytes for at most nseg segments holding at most
// `bytes` bytes in all (what a caller reserves so that later launches allocate nothing).
size_t plan_split_blob_max(uint64_t nseg, uint64_t bytes, uint64_t tile, uint32_t max_grid);
// Static launches whose chunks wait for decisions made in the same launch at lag 0: each
// segment is cut into one slice per workgroup (whole 16 KiB steps), and workgroup w takes
// slice w of every segment, in segment order.  Every chunk is then counted by the whole
// grid at once, with no tile counter, and a workgroup's next slice is loading while it waits
// for that chunk's decision.  Needs every workgroup of the launch resident (the half-CU rule
// for launches that may wait).  Tiles of one segment are not contiguous; tile0 is unused.
hist_status_t plan_striped(std::vector<SegDesc> &segs, uint32_t max_grid, MultiPlan *mp);
// own: a dedicated scratch (already sized, descriptors already on the device) or nullptr;
// either way one that only launches on `s` use.  done: as for launch_hist.  in_place: a
// device-visible copy of mp.blob that the launch reads where it is (no upload), which the
// caller keeps unchanged until the launch has finished; nullptr: the scratch's descriptors.
hist_status_t run_multi(DevCtx *d, Params &P, const MultiPlan &mp, uint32_t copies, hipStream_t s, Scratch *own,
                        bool dynamic, bool upload, hipEvent_t done = nullptr, const uint8_t *in_place = nullptr);

// Device-resident stream states: allocation and release.
struct StreamAlloc {
  StreamDev *d_st = nullptr;
  uint32_t R = 1;                 // histogram ring slots per stream
  uint64_t *d_ring = nullptr;
  Decision *d_slots = nullptr;
  uint8_t *d_mode_trace = nullptr;    // [count][trace_cap] modes, then [count][trace_cap] alarms
  uint32_t *d_pat_trace = nullptr;
  uint64_t *d_time_trace = nullptr;   // [count][trace_cap][3], all ones until written
};
hist_status_t stream_state_alloc(uint32_t count, uint32_t W, uint32_t theta, uint32_t S, uint32_t rmax, uint32_t lag,
                                 uint32_t nslot, uint32_t trace_cap, uint32_t alarm_pct, StreamAlloc *sa);
void stream_state_free(StreamAlloc *sa);

}  // namespace rt
}  // namespace histmi
