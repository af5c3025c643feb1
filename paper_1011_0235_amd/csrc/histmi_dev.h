// Internal layout shared by the HIP kernels and the host runtime of libhistmi.
#pragma once

#include <stdint.h>

#include "histmi.h"

namespace histmi {

constexpr uint32_t kBlock = 256;            // threads per workgroup (4 wavefronts of 64)
constexpr uint32_t kWaves = kBlock / 64;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kMaxCopiesLog2 = 6;      // at most 64 partial copies per segment

// How a workgroup lays out its LDS counting table for one segment.
enum Kind : uint32_t {
  KIND_WAVE = 0,      // one 256-bin table per wavefront (NVHist style)
  KIND_UNIFORM = 1,   // every value has r = 2^lg sub-bins at v*r + (lane mod r)
  KIND_LOOKUP = 2,    // per-value (base, r) from a binning pattern, via a lane-replicated index table
  KIND_WAVE_AGG = 3   // per-wavefront tables; lanes holding the same value as the first lane merge their adds
};

// A stream's kernel choice for one chunk: written by the epilogue of the chunk it was
// derived from, read by the chunk that runs with it.
struct Decision {
  uint32_t words[256];   // binning pattern words (hist_pattern_t encoding); stored only when a
                         // chunk needs them (a lookup table, or a traced chunk): a uniform
                         // pattern's words follow from the tag (value v at v << lg)
  uint32_t hist[256];    // histogram of the producing chunk (W = 1 only: the moving window)
  uint32_t S, rmax;      // stored with the words
  // stored last, in one 64-bit store, so that one load both says whether the decision is
  // there and carries what a uniform table needs:
  //   bits [32,64) producing chunk index + 1 (0: none yet), [16,24) mode (HIST_MODE_*),
  //   [0,16) table kind of the pattern (KIND_UNIFORM or KIND_LOOKUP) << 8 | log2 r if uniform
  uint64_t tag;
};
__host__ __device__ constexpr uint64_t make_tag(uint64_t gen, uint32_t mode, uint32_t kind_lg) {
  return (gen << 32) | ((uint64_t)(mode & 0xFFu) << 16) | (kind_lg & 0xFFFFu);
}
__host__ __device__ constexpr uint32_t tag_gen(uint64_t tag) { return (uint32_t)(tag >> 32); }
__host__ __device__ constexpr uint32_t tag_mode(uint64_t tag) { return (uint32_t)(tag >> 16) & 0xFFu; }
__host__ __device__ constexpr uint32_t tag_kind_lg(uint64_t tag) { return (uint32_t)tag & 0xFFFFu; }

// Size-ring entries: a chunk of a stream is a device buffer, so its size fits in 40 bits
// (1 TiB); the 24 bits above carry its generation (chunk index + 1, modulo 2^24; ring slots
// are reused every R < 2^24 chunks, so an old entry never passes for a new one).
constexpr uint32_t kSizeBits = 40;
constexpr uint64_t kSizeMask = (1ull << kSizeBits) - 1;
constexpr uint32_t kSizeGenMask = 0xFFFFFFu;

// Device-resident state of one stream (Accumulator, moving window, decisions, traces).
struct StreamDev {
  uint32_t W, theta, S, rmax, lag, nslot, trace_cap, lookup_rr;
  uint32_t R;            // sequenced streams: histogram ring slots
  uint32_t seq_lock;     // sequenced streams: 1 while a workgroup sequences chunks
  uint32_t alarm_pct;    // change detection threshold (0 = off)
  uint32_t pad;
  // A stream is sequenced (its chunks taken in order by the device) when W > 1 or alarms
  // are on; otherwise every chunk's epilogue decides on its own.
  uint64_t done;         // unsequenced: chunk epilogues completed (counted); sequenced: chunks sequenced
  uint64_t win_n;        // sequenced: bytes in the moving window after the last sequenced chunk
  uint64_t acc[256];     // Accumulator (every chunk's finalizer adds its histogram)
  uint64_t mw[256];      // sequenced: moving window after the last sequenced chunk
  // change detection (sequenced): the Accumulator in chunk order, its bytes, and the alarms
  uint64_t sacc[256];
  uint64_t sacc_n;
  uint64_t alarms, first_alarm, last_alarm;   // count; chunk index + 1 (0 = none)
  // bounded waits of this stream's chunks that gave up: a decision wait (the chunk then ran
  // the per-wavefront kernel; its trace entry is not the rule's) or a merge (the chunk's
  // histogram may be short); reported to the caller by hist_stream_read
  uint64_t wait_timeouts, merge_timeouts;
  uint64_t *ring;        // [R][256] recent histograms (sequenced), chunk j in slot j % R, each
                         // entry (j + 1) << 32 | count: a load tells whether it is chunk j's
  uint64_t *ring_n;      // [R] the same chunks' sizes, (j + 1 mod 2^24) << 40 | bytes
  Decision *slots;       // [nslot]; decision made after chunk j lives in slot j % nslot
  uint8_t *mode_trace;   // [trace_cap]
  uint8_t *alarm_trace;  // [trace_cap] 1 iff an alarm was raised after chunk k
  uint32_t *pat_trace;   // [trace_cap][256]
};

// One input buffer of a launch.
struct SegDesc {
  const uint8_t *ptr;
  uint64_t size;
  uint32_t *out;         // uint32[256] overwritten with the histogram, or null
  uint64_t *acc;         // uint64[256] the histogram is added to, or null
  int64_t chunk;         // >= 0: stream chunk index relative to Params::chunk_base; kServerChunk: server request; -1: none
  uint32_t tile0;        // first tile (launch-global index)
  uint32_t ntiles;       // >= 1 (an empty buffer still has one empty tile so it gets finalized)
  uint32_t stream_idx;   // index into Params::st for stream chunks and server requests
  uint32_t known;        // ordered-stream chunk: the decision it runs with when the host can
                         // tell it in advance (kKnown | mode << 16 | kind_lg, plus kKnownCold
                         // when there is no history yet), else 0: wait for the device's decision.
                         // kUnwalked: a window stream's chunk whose launch does not walk the
                         // window in order; kAfterAhist then gives the decision after it.
                         // kWalkAfter: a chunk whose launch leaves the in-order walk to a
                         // walk_kernel launch that follows it.
};

constexpr int64_t kServerChunk = -2;
constexpr uint32_t kKnown = 1u << 31;
constexpr uint32_t kKnownCold = 1u << 30;
constexpr uint32_t kUnwalked = 1u << 29;
constexpr uint32_t kAfterAhist = 1u << 28;
constexpr uint32_t kWalkAfter = 1u << 27;

// One tile of a multi-segment launch, written by the host: its bytes and its segment.
// Tiles never span segments; their sizes may differ (smaller tiles near the end of a
// launch shorten the tail).
struct TileRec {
  uint64_t addr;         // first byte
  uint32_t len;          // bytes (0 for the single tile of an empty segment)
  uint32_t seg;          // index into Params::segs
};

// Where a workgroup of a static launch starts: its tile range, its first tile and that
// tile's segment, in one record, so that starting costs one memory round trip instead of
// three dependent ones (tile range, then tile, then segment).
struct WgStart {
  uint32_t tile, tile_end;   // tiles [tile, tile_end) (empty when equal)
  TileRec first;             // tile `tile` (zero if none)
  SegDesc seg;               // its segment's descriptor
};
constexpr uint32_t kStartWords = sizeof(WgStart) / 4;
static_assert(sizeof(WgStart) % 4 == 0 && kStartWords <= 64, "one word per lane of the first wavefront");

// Kernel arguments.  Every field a launch reads is in the first five 64-byte lines (the
// kernel touches all five at entry, so that their scalar-cache misses overlap instead of
// following one another); the 1 KiB of host pattern words, read only by lookup-table
// launches, comes last.
struct Params {
  // line 0: the launch's shape and LDS layout (32-bit fields)
  uint32_t single;           // 1: one buffer described by seg0, spread over the whole grid
  uint32_t dynamic;          // 1: tiles handed out in order by an atomic counter; 0: static
  uint32_t nseg;
  uint32_t ntiles;
  uint32_t clog2;            // log2 of the partial copies per segment
  uint32_t table_words;      // LDS layout (in 32-bit words): counting table at word 0
  uint32_t look_off;         // lane-replicated lookup table (byte addresses into the counting table)
  uint32_t look_words;
  // non-stream segments: one kind for every segment
  uint32_t kind;             // Kind
  uint32_t uni_lg;           // KIND_UNIFORM: log2 r
  uint32_t pat_S;            // KIND_LOOKUP: pattern size; stream launches: counting-table capacity
  uint32_t look_rr_lg;       // log2 of the lookup replication (5 or 6)
  uint32_t forced;           // stream chunks: 0 = decided per chunk, else HIST_MODE_AHIST / HIST_MODE_WAVEHIST
  uint32_t ordered;          // 1 for an ordered stream launch (one stream, segment j is chunk chunk_base + j)
  // bounded waits: polls of a decision tag, and re-reads of a segment's partial copies,
  // before they give up (counted in the diagnostics and the stream's state)
  uint32_t wait_polls;
  uint32_t merge_polls;
  // line 1
  SegDesc seg0;              // the descriptor when single
  // lines 1-3: device arrays
  const SegDesc *segs;       // device array of nseg descriptors (unused when single)
  const TileRec *recs;       // [ntiles] tiles in launch order (unused when single)
  const uint32_t *bounds;    // [grid + 1] static launches: workgroup g takes tiles [bounds[g], bounds[g+1])
  const WgStart *starts;     // [grid] static launches: each workgroup's start record
  uint32_t *ctr;             // [0] next tile, [1] workgroups finished (both reset by the last one)
  uint32_t *seg_done;        // [nseg] tiles finished per segment (reset by the finalizer)
  uint32_t *partial;         // [nseg][copies][256] partial counts (reset by the finalizer)
  uint32_t *diag;            // device diagnostics counters
  StreamDev *st;             // stream chunks and server requests: array of stream states
  Decision *slots;           // ordered launches: the stream's decision ring
  uint64_t *time_trace;      // [trace_cap][3] per traced chunk: device wall-clock ticks when its
                             // first workgroup began counting it (atomic min) and when its
                             // finalizer was done (decision ready; W > 1: histogram in the ring),
                             // and the cycle counter's rate (ticks per us) inside that finalizer
  uint64_t chunk_base;       // absolute index of relative chunk 0
  uint64_t trace_cap;
  // line 4: copies of an ordered stream's constants, so that starting a chunk reads nothing
  // but its decision's tag
  uint32_t lag;
  uint32_t nslot;
  uint32_t W;                // moving-window length in chunks
  uint32_t theta;            // critical degeneracy, percent
  uint32_t S;                // sub-bin budget of rule P
  uint32_t rmax;             // sub-bin cap of rule P
  uint32_t R;                // histogram ring slots (sequenced streams)
  uint32_t alarm_pct;        // change detection threshold (0 = off); sequenced when W > 1 or on
  uint32_t criterion;        // HIST_CRIT_*
  uint32_t kappa;            // collision-index threshold, percent
  // single-buffer launches: when set, the finalizer stores done_seq here (pinned host memory,
  // system scope) once the histogram and every state update are visible to the host and to
  // other engines, so the host sees completion without an event
  uint32_t done_seq;
  uint32_t *host_done;
  // read only by launches with a host pattern (KIND_LOOKUP)
  uint32_t pat_words[256];
};
constexpr uint32_t kHotParamLines = 5;


// Launch configuration chosen by the host.
struct LaunchShape {
  uint32_t grid;
  uint32_t lds_bytes;
  uint32_t unroll;
};

}  // namespace histmi
