/*
 * histmi -- exact 256-bin histograms of packed 8-bit pixel streams on MI355X (gfx950).
 *
 * C ABI of libhistmi.so.  The operations follow Koppaka et al., "Fast Histograms
 * using Adaptive CUDA Streams" (2010):
 *   - the histogram itself: 256 counts of byte values 0..255, exact (Sec. I, Sec. III.A);
 *   - AHist: each value's atomics spread over r sub-bins of an on-chip sub-histogram,
 *     assigned to the lanes of a wavefront cyclically, indexed by a binning pattern
 *     (Sec. III.A, Figure 1, discussion of Table 2);
 *   - the per-wavefront sub-histogram kernel the paper compares against (NVHist, Sec. I,
 *     Table 2), here one 256-bin table per 64-lane wavefront;
 *   - streams with an Accumulator and a moving-window (MW) histogram, the pattern
 *     recomputed from past histograms, and a kernel switch on the degeneracy of the
 *     last MW histogram (Sec. III.B, Sec. III.C);
 *   - many slices batched into one asynchronous call returning many histograms
 *     (Sec. III.B).
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device memory of the current HIP device; h_* are host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *     enqueued asynchronously on it unless the description says "synchronous".
 *   - The caller owns every input and output buffer.  The library owns opaque handles,
 *     their device state and its internal scratch.
 *   - Calls return a status and never abort or throw.  Argument errors are returned
 *     synchronously and enqueue nothing.  Errors of the HIP runtime map to HIST_EDEVICE.
 *   - A handle is used by one host thread at a time, except hist_server_submit/poll,
 *     which are thread-safe.
 *   - Counts never depend on the mode or the binning pattern: every mode and every valid
 *     pattern give the identical histogram.
 */
#ifndef HISTMI_H
#define HISTMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HIST_OK = 0,
    HIST_EINVAL = -1,     /* bad argument: NULL buffer with n > 0, bad mode, invalid pattern, ... */
    HIST_ENOMEM = -2,     /* device or host allocation failed */
    HIST_EOVERFLOW = -3,  /* a count could exceed its 32-bit output (n >= 2^32 for hist_u8) */
    HIST_EBUSY = -4,      /* server queue full */
    HIST_EDEVICE = -5,    /* the HIP runtime reported an error */
    HIST_ENOTSUP = -6,    /* not supported on this device (e.g. not gfx950) */
    HIST_ETIMEDOUT = -7,  /* a wait ran out of time */
    HIST_ECANCELED = -8   /* request canceled (server shut down before it ran) */
} hist_status_t;

typedef enum {
    /* hist_u8 / hist_u8_u64 / hist_batch: the kernel the library measured fastest for a
     * call with no history (lane-cyclic sub-bins, HIST_AUTO_FLAT_R per value).
     * Streams and the server: the paper's switch (Sec. III.C) -- AHist with the pattern
     * derived from the moving window when the window is degenerate, else per-wavefront. */
    HIST_MODE_AUTO = 0,
    HIST_MODE_AHIST = 1,     /* sub-bins indexed by the binning pattern */
    HIST_MODE_WAVEHIST = 2,  /* one 256-bin table per wavefront (NVHist style) */
    HIST_MODE_WAVEAGG = 3    /* per-wavefront tables; per byte position, the lanes whose value equals the
                                first active lane's are merged into one add of their count (64-lane ballot) */
} hist_mode_t;

typedef enum {
    HIST_PAT_IDENTITY = 0,   /* r = 1 for every value, base = value (S = 256) */
    HIST_PAT_PAPER960 = 1,   /* reconstruction of Figure 1: runs of 32 values, r = 1,2,4,8,8,4,2,1 (S = 960) */
    HIST_PAT_FLAT = 2        /* r = rmax for every value, in value order (S = 256 * rmax) */
} hist_pattern_kind_t;

#define HIST_BINS 256
#define HIST_S_MAX 16384u        /* largest sub-histogram (sub-bins) a pattern may use */
#define HIST_RMAX_MAX 64u        /* most sub-bins per value: one per lane of a wavefront */
#define HIST_AUTO_FLAT_R 32u     /* sub-bins per value used by HIST_MODE_AUTO for history-free calls */

/*
 * Binning pattern (Sec. III.A: 256 entries that index a value's bins in the shared
 * sub-histogram; Figure 1).  word[v]: bits [0,16) = base sub-bin of value v,
 * bits [16,24) = log2 r(v), bits [24,32) = 0.  Lane L of a wavefront adds value v into
 * sub-bin base(v) + (L mod r(v)) (cyclic allotment of sub-bins to lanes, discussion of
 * Table 2).  Valid iff rmax is a power of two in [1, HIST_RMAX_MAX], every r(v) is a
 * power of two <= rmax, total_S <= HIST_S_MAX, every range [base, base + r) lies inside
 * [0, total_S), and the 256 ranges are pairwise disjoint.  1032 bytes; may live in host
 * or device memory as each call states.
 */
typedef struct {
    uint32_t word[256];
    uint32_t total_S;
    uint32_t rmax;
} hist_pattern_t;

const char *hist_strerror(hist_status_t e);

/* Device facts the library sees (synchronous).  arch: e.g. "gfx950". */
typedef struct {
    int device;
    int cu_count;
    int clock_khz;
    size_t lds_per_cu;
    size_t hbm_bytes;
    char arch[32];
} hist_device_info_t;
hist_status_t hist_device_info(hist_device_info_t *info);

/*
 * hist_u8 -- out[b] = #{ i < n : in[i] == b } for b = 0..255 (Sec. III.A; exact, Sec. I).
 *   d_in:   n bytes of device memory, any alignment (n = 0: d_in may be NULL).
 *   d_out:  device uint32[256], OVERWRITTEN (n = 0 gives zeros).
 *   mode:   HIST_MODE_AUTO / AHIST / WAVEHIST.
 *   h_pat:  HOST hist_pattern_t used by HIST_MODE_AHIST (NULL = HIST_PAT_IDENTITY); it is
 *           checked on the host and copied into the launch, so it may be freed on return.
 *           Ignored by the other modes.
 * Errors: HIST_EINVAL (NULL d_in with n > 0, NULL d_out, bad mode, invalid pattern),
 *         HIST_EOVERFLOW (n >= 2^32: use hist_u8_u64), HIST_EDEVICE.
 */
hist_status_t hist_u8(const void *d_in, size_t n_bytes, uint32_t *d_out, hist_mode_t mode,
                      const hist_pattern_t *h_pat, void *stream);

/* hist_u8_u64 -- as hist_u8 but ACCUMULATES into device uint64[256] d_acc; any n. */
hist_status_t hist_u8_u64(const void *d_in, size_t n_bytes, uint64_t *d_acc, hist_mode_t mode,
                          const hist_pattern_t *h_pat, void *stream);

/*
 * hist_u8_noalloc -- hist_u8 for callers that cannot allocate device memory: code under
 * HIP graph capture, serving loops and harnesses that forbid hipMalloc.  Same arguments,
 * result and errors as hist_u8, and the same counting kernel; it calls no hipMalloc or
 * hipFree, not even on its first call.  Its scratch (counters and partial histograms) is a
 * fixed array of HIST_NOALLOC_SCRATCH_BYTES compiled into the library; each device the
 * library runs on holds its own copy until the process ends.  Each call clears what it
 * needs of it with a small kernel on `stream` (no memset), then launches the histogram.
 * All calls on one device share that array: calls that overlap on the device (on
 * different HIP streams without ordering between them, or from several host threads) race
 * and may return wrong counts; order them.
 * Extra error: HIST_ENOMEM if a launch would need more scratch than the array holds (not
 * reached at the library's launch shapes: at most 16 partial copies of 1 KiB).
 */
#define HIST_NOALLOC_SCRATCH_BYTES 32768u
hist_status_t hist_u8_noalloc(const void *d_in, size_t n_bytes, uint32_t *d_out, hist_mode_t mode,
                              const hist_pattern_t *h_pat, void *stream);

/* hist_pattern_init -- fill a HOST pattern of the given kind (synchronous).
 *   IDENTITY ignores S/rmax (S = 256, rmax = 1); PAPER960 ignores them (S = 960, rmax = 8);
 *   FLAT needs rmax a power of two <= HIST_RMAX_MAX (S = 256 * rmax; the S argument is ignored). */
hist_status_t hist_pattern_init(hist_pattern_t *h_pat, hist_pattern_kind_t kind, uint32_t S, uint32_t rmax);

/* hist_pattern_validate -- HIST_OK iff the HOST pattern is valid (see hist_pattern_t). */
hist_status_t hist_pattern_validate(const hist_pattern_t *h_pat);

/*
 * hist_pattern_update -- recompute the pattern from a past histogram (Sec. III.B: the
 * indices are recomputed from the past stream's histograms).  The paper gives no rule;
 * this is rule P: with N = sum h, if 256*rmax <= S every value gets rmax; else if N = 0
 * every value gets 1; else r_t(v) = min(rmax, pow2ceil(max(1, ceil(h(v) 2^t / N)))) for the
 * largest t in [0, min(24, 64 - bitlen(N))] with sum_v r_t(v) <= S, laid out by
 * (r descending, value ascending) with bases as running sums.
 *   d_hist: device uint64[256];  d_pat: device hist_pattern_t, overwritten.
 *   Needs 256 <= S <= HIST_S_MAX and rmax a power of two <= HIST_RMAX_MAX, else HIST_EINVAL.
 */
hist_status_t hist_pattern_update(const uint64_t *d_hist, uint32_t S, uint32_t rmax, hist_pattern_t *d_pat,
                                  void *stream);

/* ---------------------------------------------------------------- streams (Sec. III.B, III.C) */

typedef struct hist_stream hist_stream_t;

typedef struct {
    uint32_t W;          /* moving window length in chunks, >= 1 (Table 4 uses 32, 128, 256) */
    uint32_t theta_pct;  /* critical degeneracy in percent, 0..100 (Sec. III.C: 40-50) */
    uint32_t S;          /* sub-histogram budget for rule P, 256..HIST_S_MAX */
    uint32_t rmax;       /* most sub-bins per value, power of two <= HIST_RMAX_MAX */
    uint32_t lag;        /* chunk k runs with the decision made after chunk k-1-lag (0 = sequential) */
    uint32_t trace_cap;  /* chunks whose (mode, pattern, alarm) are recorded for hist_stream_read */
    uint32_t alarm_pct;  /* change detection (see below): 0 = off, else 1..100 percentage points */
    uint32_t criterion;  /* switching test: HIST_CRIT_MAXBIN (the paper's, default), _COLLISION, _BOTH */
    uint32_t kappa_pct;  /* collision-index threshold in percent, 0..100 (HIST_CRIT_COLLISION / _BOTH) */
} hist_stream_config_t;

/* Switching criteria.  MAXBIN is the paper's degeneracy test (Sec. III.C).  COLLISION is an
 * alternative (the paper leaves other criteria to future work, naming one that measures the
 * serialisation the data would cause; this is the library's reading): the window's collision
 * index sum_v p_v^2, the probability that two lanes of a wavefront add into the same bin,
 * tested as 100 * sum_v MW(v)^2 > kappa * (sum_v MW(v))^2 in exact integers.  BOTH takes AHist
 * when either test does. */
#define HIST_CRIT_MAXBIN 0u
#define HIST_CRIT_COLLISION 1u
#define HIST_CRIT_BOTH 2u

/*
 * Stream semantics.  Chunk k gets histogram h_k.  After chunk k the device updates
 *   Acc += h_k (uint64, the Accumulator), MW = h_{k-W+1} + ... + h_k (the moving window),
 *   D_k = (AHIST if 100 * max_v MW(v) > theta * sum_v MW(v) else WAVEHIST, rule P(MW))
 * (with the MAXBIN criterion; see HIST_CRIT_* for the others).
 * Chunk k runs with D_{k-1-lag}; chunks with k-1-lag < 0 run WAVEHIST with the identity
 * pattern.  A forced mode in push replaces the decided kernel but not the pattern.  All
 * state lives on the device; no host round trip happens between chunks.
 *
 * Change detection (Sec. III.B proposes comparing the moving window, the stream's present,
 * with the Accumulator, its general nature, to detect an attack or a need to reprocess; the
 * measure is this library's reading): with alarm_pct > 0 the device raises an alarm after
 * chunk k iff some value v's share of MW differs from its share of Acc by more than
 * alarm_pct percentage points, i.e. 100 * |MW(v) * sum Acc - Acc(v) * sum MW| >
 * alarm_pct * sum MW * sum Acc (exact integers; never with an empty MW or Acc; exact while
 * the Accumulator holds fewer than 2^60 bytes).  A stream with alarms on is sequenced in
 * chunk order on the device (as every stream with W > 1 is).  When every decision is a
 * function of the chunk sizes (a budget of rmax sub-bins for every value, and theta or kappa
 * 0), the host hands each chunk its decision: a stream with alarms then walks its chunks in
 * order in a one-workgroup launch queued after each push, and a window stream without
 * alarms does not walk them at all (its window is summed from its ring of recent
 * histograms when read).  The results are the same either way.
 *
 * Pushes of one stream must be issued from one host thread at a time, in chunk order, but
 * may go to different HIP streams: a chunk waits on the device for the decision it runs
 * with, so consecutive launches may overlap (the tail of one filling the device while the
 * next starts) and the results do not depend on timing.  At most two launches of one stream
 * are in flight: a push makes its HIP stream wait for the launch two before it.  A HIP
 * stream given to a push must stay valid until the next hist_stream_read (or
 * hist_stream_read_alarms, hist_stream_destroy) returns: those wait for it, and a later
 * push on another HIP stream may queue an event on it.
 */
hist_status_t hist_stream_create(hist_stream_t **st, const hist_stream_config_t *cfg);

/* One chunk.  d_out_k: device uint32[256] overwritten with h_k, or NULL. */
hist_status_t hist_stream_push(hist_stream_t *st, const void *d_chunk, size_t n, hist_mode_t mode,
                               uint32_t *d_out_k, void *stream);

/* Many chunks in one persistent launch (same semantics as `count` pushes).
 * h_ptrs/h_sizes: HOST arrays of device pointers and sizes (< 2^32 each).
 * d_out: device uint32[count][256] (row k overwritten with h_k), or NULL. */
hist_status_t hist_stream_push_many(hist_stream_t *st, const void *const *h_ptrs, const uint64_t *h_sizes,
                                    uint32_t count, hist_mode_t mode, uint32_t *d_out, void *stream);

typedef struct {
    uint64_t chunks;       /* chunks pushed so far */
    uint64_t acc[256];     /* Accumulator */
    uint64_t mw[256];      /* moving window after the last chunk */
    uint32_t next_mode;    /* decided kernel after the last chunk (HIST_MODE_AHIST / WAVEHIST) */
    hist_pattern_t next_pattern;  /* rule P of the current moving window */
    uint64_t alarms;       /* change detection: chunks after which an alarm was raised */
    uint64_t first_alarm;  /* index + 1 of the first such chunk, 0 if none */
    uint64_t last_alarm;   /* index + 1 of the last such chunk, 0 if none */
    uint64_t wait_timeouts;   /* chunks whose bounded wait for their decision gave up (they ran the
                                 per-wavefront kernel: counts exact, trace entry not the rule's) */
    uint64_t merge_timeouts;  /* chunks whose merge gave up before its total arrived (histogram may be short) */
} hist_stream_snapshot_t;

/* Synchronous: waits for `stream` and for this stream's launches on any HIP stream, then
 * copies the state.  A window stream whose pushes did not walk the window (see
 * hist_stream_create) first has it summed from its ring by a one-workgroup launch on
 * `stream`, which this call also waits for.  h_mode_trace (uint8[trace_len])
 * and h_pattern_trace (uint32[trace_len][256]) may be NULL; entry k holds the mode / pattern
 * words chunk k ran with (k < trace_cap).
 * Returns HIST_ETIMEDOUT, with everything still copied, when a bounded wait of one of the
 * stream's chunks gave up (see wait_timeouts and merge_timeouts; never expected at the
 * default limits, see hist_set_wait_limits).  The Accumulator, the moving window and the chunk
 * count stay exact after a decision wait gave up; only that chunk's trace entry differs. */
hist_status_t hist_stream_read(hist_stream_t *st, hist_stream_snapshot_t *snap, uint8_t *h_mode_trace,
                               uint32_t *h_pattern_trace, uint32_t trace_len, void *stream);

/* Change detection trace (Sec. III.B).  Synchronous like hist_stream_read.  h_alarm_trace:
 * HOST uint8[trace_len]; entry k is 1 iff an alarm was raised after chunk k (k < trace_cap;
 * entries of chunks not yet pushed are 0).  HIST_EINVAL if the stream has alarms off or
 * h_alarm_trace is NULL with trace_len > 0. */
hist_status_t hist_stream_read_alarms(hist_stream_t *st, uint8_t *h_alarm_trace, uint32_t trace_len, void *stream);

/* Per-chunk timeline of the device, for the chunks of the trace (the per-chunk breakdown of
 * a stream's time behind Sec. III.B's pipelining: how long each chunk waits for its decision
 * and how long it takes).  Synchronous like hist_stream_read.  h_times_ns: HOST
 * uint64[trace_len][3]; entry k = {the time the first workgroup began counting chunk k
 * (after its decision arrived), the time chunk k's decision was ready (with W > 1 or change
 * detection: its histogram handed to the in-order sequencer), the rate of the shader's
 * cycle counter (s_memtime) in ticks per microsecond measured inside chunk k's finalizer,
 * which follows the engine clock}; times in nanoseconds of the device's constant-rate
 * wall clock (differences are meaningful, the origin is not).  0 for chunks beyond
 * trace_cap or not yet run.  HIST_EINVAL if h_times_ns is NULL with trace_len > 0. */
hist_status_t hist_stream_read_times(hist_stream_t *st, uint64_t *h_times_ns, uint32_t trace_len, void *stream);

/* Synchronous; waits for the device before freeing. */
hist_status_t hist_stream_destroy(hist_stream_t *st);

/* ---------------------------------------------------------------- host ingest (Sec. III.B) */

/*
 * Streams whose chunks live in HOST memory: each chunk is copied to the device and pushed
 * through a stream, with the copies of some chunks overlapping the counting of others across
 * n_hip_streams HIP streams -- the paper's pipelined stream (Sec. III.B, Fig. 2), whose
 * benefit it measures against 1..256 CUDA streams (Figs. 3-4).  The decisions stay on the
 * device, so no host round trip is needed between chunks.  Calling hist_ingest_sync after
 * every push gives the sequential variant the paper compares against.
 */
typedef struct hist_ingest hist_ingest_t;

typedef struct {
    uint32_t n_hip_streams;   /* 1..256 HIP streams used in turn */
    uint64_t slot_bytes;      /* largest chunk (< 2^32); one device staging buffer of this size per HIP stream */
} hist_ingest_config_t;

hist_status_t hist_ingest_create(hist_ingest_t **ing, const hist_ingest_config_t *cfg);

/* Copies h_chunk[0, n) (host memory; pinned memory, e.g. from hipHostMalloc, copies at full
 * speed and asynchronously) into the next HIP stream's staging buffer and pushes it as one
 * chunk of `st` (the semantics of hist_stream_push).  Returns once the copy and the launch
 * are queued: h_chunk must stay valid and unchanged until hist_ingest_sync returns.
 * d_out_k: device uint32[256] overwritten with the chunk's histogram, or NULL.
 * Errors: HIST_EINVAL (NULL handles, NULL h_chunk with n > 0, n > slot_bytes, bad mode). */
hist_status_t hist_ingest_push(hist_ingest_t *ing, hist_stream_t *st, const void *h_chunk, size_t n,
                               hist_mode_t mode, uint32_t *d_out_k);

/* Waits for every queued copy and launch of this ingest. */
hist_status_t hist_ingest_sync(hist_ingest_t *ing);

/* Synchronous; waits before freeing. */
hist_status_t hist_ingest_destroy(hist_ingest_t *ing);

/* ---------------------------------------------------------------- batches (Sec. III.B) */

/*
 * hist_batch -- n histograms in one persistent launch.
 *   h_ptrs, h_sizes: HOST arrays of n device pointers (any alignment) and sizes (< 2^32).
 *   d_out: device uint32[n][256]; row j OVERWRITTEN with the histogram of buffer j.
 *   mode, h_pat: as for hist_u8, one choice for all n buffers.
 */
hist_status_t hist_batch(const void *const *h_ptrs, const uint64_t *h_sizes, uint32_t n, uint32_t *d_out,
                         hist_mode_t mode, const hist_pattern_t *h_pat, void *stream);

/* A batch captured once into a HIP graph (descriptors uploaded at create time); each launch
 * recomputes all n histograms from the current contents of the same buffers. */
typedef struct hist_batch_graph hist_batch_graph_t;
hist_status_t hist_batch_graph_create(hist_batch_graph_t **g, const void *const *h_ptrs, const uint64_t *h_sizes,
                                      uint32_t n, uint32_t *d_out, hist_mode_t mode, const hist_pattern_t *h_pat);
hist_status_t hist_batch_graph_launch(hist_batch_graph_t *g, void *stream);
hist_status_t hist_batch_graph_destroy(hist_batch_graph_t *g);

/* ---------------------------------------------------------------- served requests */

/*
 * A continuous-batching server of histogram requests.  Requests carry a stream id; each
 * stream id has device-resident state: a uint64 running histogram and the kernel decision
 * (mode and binning pattern) recomputed from its latest finished request with the paper's
 * switch (Sec. III.C) and rule P (the pattern from past histograms, Sec. III.B).  A scheduler
 * thread admits queued requests in arrival order while the admitted bytes stay within the
 * HBM budget and the admitted requests within max_slots, packs them into micro-batches (one
 * persistent launch each, as hist_batch; the paper batches small slices into one asynchronous
 * call, Sec. III.B) and spreads the micro-batches over n_hip_streams HIP streams, so work
 * admitted while other batches run overlaps with them on the device.
 *
 * Each request's histogram is exact and does not depend on what else is in flight; a
 * stream's running histogram is the order-free sum of its finished requests.  A stream's
 * decision follows its latest finished request (a window of one request), so which kernel a
 * request runs with depends on timing -- only speed does.
 */
typedef struct hist_server hist_server_t;

typedef struct {
    uint64_t hbm_budget_bytes;  /* bytes of admitted, unfinished requests, at most (> 0) */
    uint32_t max_slots;         /* admitted, unfinished requests, at most (>= 1) */
    uint32_t n_stream_ids;      /* stream ids 0..n-1 (1..65536) */
    uint32_t n_hip_streams;     /* HIP streams the micro-batches are spread over (1..16) */
    uint32_t max_batch;         /* requests per micro-batch, at most (>= 1) */
    uint32_t mode;              /* hist_mode_t: AUTO = per-stream decision; AHIST / WAVEHIST forced */
    uint32_t theta_pct;         /* critical degeneracy, percent */
    uint32_t S;                 /* sub-histogram budget for rule P (256..HIST_S_MAX) */
    uint32_t rmax;              /* most sub-bins per value (power of two <= HIST_RMAX_MAX) */
    uint32_t idle_spin_us;      /* the scheduler spins this long after its last activity before it
                                   blocks (0: 20000; at most 10^7).  A submission to a blocked
                                   scheduler waits 10-25 us for its wake-up; spinning costs a core */
} hist_server_config_t;

typedef struct {
    int32_t status;             /* HIST_OK finished; HIST_EBUSY queued or running; HIST_ECANCELED; HIST_EDEVICE */
    uint32_t stream_id;
    uint64_t bytes;
    uint64_t t_submit_ns;       /* CLOCK_MONOTONIC: submit returned the ticket */
    uint64_t t_admit_ns;        /* admitted into a micro-batch (0 if not yet) */
    uint64_t t_done_ns;         /* the host saw the micro-batch finish (0 if not yet) */
} hist_server_result_t;

typedef struct {
    uint64_t submitted, completed, canceled, batches, bytes_done;
    uint64_t max_inflight_bytes, max_inflight_requests, max_concurrent_batches;
    uint64_t max_launch_ns;      /* longest host call that queued one micro-batch (HIP launch path) */
    uint64_t max_query_ns;       /* longest host call that asked whether a micro-batch had finished */
} hist_server_stats_t;

/* Synchronous.  Starts the scheduler thread on the current device.  The scheduler spins on
 * one host core while micro-batches are in flight and for idle_spin_us after its last
 * activity (a timed sleep would round up to the OS timer slack and set the latency floor);
 * idle beyond that it blocks until the next submission.  Everything a micro-batch of up to
 * min(max_batch, max_slots, 1024) requests needs is allocated here, per slot: device scratch
 * and a pinned host buffer of descriptors that the kernel reads in place, so the scheduler's
 * launches neither allocate nor copy (a larger batch grows its slot's scratch on first use). */
hist_status_t hist_server_create(hist_server_t **sv, const hist_server_config_t *cfg);

/* Thread-safe, non-blocking.  d_buf: n device bytes (any alignment) that stay unchanged until
 * the request finishes; d_out: device uint32[256] overwritten with the histogram (or NULL).
 * Errors: HIST_EINVAL (bad id, NULL buffer with n > 0, n above the HBM budget),
 * HIST_EOVERFLOW (n >= 2^32), HIST_EBUSY (queue of not-yet-admitted requests full),
 * HIST_ECANCELED (server shutting down). */
hist_status_t hist_server_submit(hist_server_t *sv, uint32_t stream_id, const void *d_buf, size_t n, uint32_t *d_out,
                                 uint64_t *ticket);

/* Thread-safe, non-blocking: fills r (r->status HIST_EBUSY while the request is not done).
 * A ticket is retired once poll or wait has reported its final state (a status other than
 * HIST_EBUSY); later calls with it, and calls with a ticket never issued, return HIST_EINVAL.
 * Finished tickets that nobody polls are retired oldest first once more than 2^20 of them
 * are held, so a server's host memory stays bounded. */
hist_status_t hist_server_poll(hist_server_t *sv, uint64_t ticket, hist_server_result_t *r);

/* Blocks until the request is done or timeout_ns passes (< 0: no limit); HIST_ETIMEDOUT then
 * (the ticket stays live).  r may be NULL.  Retires a finished ticket as poll does. */
hist_status_t hist_server_wait(hist_server_t *sv, uint64_t ticket, int64_t timeout_ns, hist_server_result_t *r);

/* Blocks until every submitted request is done (or timeout_ns passes: HIST_ETIMEDOUT). */
hist_status_t hist_server_drain(hist_server_t *sv, int64_t timeout_ns);

/* Synchronous copy of a stream's running uint64[256] histogram (complete after a drain). */
hist_status_t hist_server_stream_acc(hist_server_t *sv, uint32_t stream_id, uint64_t *h_acc);

hist_status_t hist_server_stats(hist_server_t *sv, hist_server_stats_t *st);

/* Cancels requests not yet admitted (HIST_ECANCELED), waits for admitted ones, frees everything. */
hist_status_t hist_server_destroy(hist_server_t *sv);

/* ---------------------------------------------------------------- diagnostics and tuning */

typedef struct {
    uint64_t invalid_patterns;   /* device-side checks of stream patterns that failed (chunk ran per-wavefront) */
    uint64_t wait_timeouts;      /* bounded in-kernel waits that gave up (stream state may be stale) */
    uint64_t merge_timeouts;     /* finalizers whose partial counts never reached the segment size */
} hist_diag_t;
/* Synchronous read of the current device's counters. */
hist_status_t hist_diag_read(hist_diag_t *d);

/*
 * hist_read_probe -- the HBM read roofline the histogram kernels are measured against: a
 * plain streaming read of n_bytes at d_in (16-byte vector loads, grid-stride, each byte read
 * once) whose little-endian uint32 words are summed and ADDED to *d_sum (device uint64).
 *   d_in: device pointer, 16-byte aligned; n_bytes: a multiple of 16 (0 is a no-op).
 *   workgroups: grid size (256 threads each), 1..65536; 0 = two per compute unit.
 * Errors (synchronous): HIST_EINVAL for NULL pointers, misaligned/ragged sizes or a grid
 * out of range.  Asynchronous on `stream`.  Not part of the histogram path: a measurement aid.
 */
hist_status_t hist_read_probe(const void *d_in, size_t n_bytes, uint64_t *d_sum, uint32_t workgroups,
                              void *stream);

/*
 * hist_set_wait_limits -- bounds of the in-kernel waits of launches issued after the call
 * (process-wide; synchronous; never fails).  decision_polls: polls of a stream chunk's
 * decision before the chunk gives up and runs the per-wavefront kernel (0 = the default,
 * 2^22, about a second); merge_polls: re-reads of a segment's partial counts before its
 * finalizer gives up (0 = the default, 2^20).  Every wait is bounded, so every kernel ends;
 * a wait that gave up is counted in hist_diag_t and in the stream's snapshot.  Small limits
 * exist to exercise those paths; they cost speed (and, for merges, exactness) only.
 */
hist_status_t hist_set_wait_limits(uint32_t decision_polls, uint32_t merge_polls);

/* Launch shape of one kernel family.  Zero fields keep the built-in default. */
typedef struct {
    uint32_t blocks_per_cu;   /* persistent workgroups per compute unit */
    uint32_t tile_kib;        /* largest tile of a multi-buffer launch in KiB (multiple of 16, 16..1048576) */
    uint32_t merge_copies;    /* partial-histogram copies a segment spreads its merge over (power of 2) */
    uint32_t tiles_per_wg;    /* multi-buffer launches: tiles are made small enough that every
                                 workgroup gets about this many (1..64); launches that never
                                 wait give each workgroup one equal share of the bytes, cut
                                 into tiles at chunk boundaries, and family 5 ignores it */
} hist_tune_t;
/* family: 0 = per-wavefront, 1 = lane-cyclic uniform sub-bins, 2 = pattern lookup,
 * 3 = wavefront aggregation (these four for hist_u8 / hist_batch / the server, by kernel),
 * 4 = ordered stream pushes whose chunks wait for the device's decisions (tiles handed out
 * in chunk order), 5 = ordered stream pushes whose decisions the host knows in advance
 * (a budget of rmax sub-bins for every value and a switching threshold of 0: nothing waits,
 * and each workgroup takes one equal share of the bytes). */
#define HIST_TUNE_STREAM 4u
#define HIST_TUNE_STREAM_KNOWN 5u
hist_status_t hist_tune_set(uint32_t family, const hist_tune_t *t);
hist_status_t hist_tune_get(uint32_t family, hist_tune_t *t);

#ifdef __cplusplus
}
#endif

#endif /* HISTMI_H */
