// HIP kernels of libhistmi for gfx950 (CDNA4, wave64).
//
// One persistent kernel family does every histogram launch.  A launch covers one or more
// segments (input buffers); each segment is cut into tiles and each workgroup takes whole
// tiles.  For every segment a workgroup touches it:
//   1. stages an LDS counting table (kind chosen per segment, see Kind);
//   2. streams its tiles with 16-byte loads (1 KiB per wavefront per load) and adds every
//      byte into the table with one ds_add_u32 (the hot loop);
//   3. sums the table down to 256 counts (one per thread) and merges them into one of
//      several partial copies of the segment's histogram in global memory with
//      no-return atomics (spread over copies so that same-address atomics do not serialize);
//   4. takes a ticket; the workgroup finishing the segment's last tile sums the copies,
//      writes the segment's histogram, resets the copies and, for a stream chunk, runs the
//      stream epilogue (Accumulator, moving window, degeneracy switch, rule P).
//
// The counting tables follow the paper's two kernels (Sec. III.A, Table 2):
//   KIND_WAVE    -- one 256-bin table per wavefront, the per-warp sub-histograms of the
//                   NVIDIA SDK kernel the paper compares against;
//   KIND_UNIFORM -- AHist with every value given r sub-bins, lane L adding into sub-bin
//                   v*r + (L mod r) (the cyclic allotment of sub-bins to the threads of a
//                   warp); with r >= 32 the 64 lanes of a wavefront never collide in a bank;
//   KIND_LOOKUP  -- AHist with an arbitrary binning pattern (Figure 1): per value a base and
//                   a power-of-two r; the lane-specific sub-bin address comes from an
//                   LDS table replicated per lane so that the lookup itself is conflict free;
//   KIND_WAVE_AGG -- per-wavefront tables, with the lanes that hold the first active lane's
//                   value merged into one add (a 64-lane ballot): another way to cut the
//                   serialised same-address atomics of peaked data.

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "histmi_dev.h"

namespace histmi {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// Global-address-space views: loads through them compile to global_load_* (vmcnt only)
// instead of flat_load_*, which would also count against the LDS wait counter.
typedef __attribute__((address_space(1))) const u32x4 gu32x4;
typedef __attribute__((address_space(1))) const uint8_t gu8;
// LDS addressed by integer byte address: the table base is folded into per-lane constants
// once, so each byte costs one extract and one shift-add before its ds_add_u32.
typedef __attribute__((address_space(3))) uint32_t lu32;
__device__ __forceinline__ uint32_t lds_addr_of(const uint32_t *p) {
  return (uint32_t)(uintptr_t)(const lu32 *)p;
}

// Small control block in static LDS.
struct Ctl {
  uint32_t next_tile;
  uint32_t flag;
  uint32_t kind;
  uint32_t lg;
  uint32_t used_mode;
  uint32_t tmp;
  uint64_t tag;            // decision tag of the current segment's stream chunk
  uint32_t sflag[2][kWaves];  // the sequencer's per-wavefront flags, by chunk parity
  uint64_t ptag[8];        // the sequencer's decision tags of one batch, published together
  uint64_t alarms[3];      // the sequencer's change-detection count, first and last alarm
  uint64_t coll[3][4][3];  // collision criterion: limb sums of sum MW^2 [batch mod 3][chunk][limb]
  // multi-segment launches, double-buffered so that one barrier per step suffices:
  SegDesc sd[2];           // the current segment's descriptor (and the next one's, being staged)
  TileRec nrec[2];         // the next tile's record, by tile parity
  uint32_t ntile[2];       // the next tile's index, by tile parity
  uint32_t start[6];       // static launches: tile range and first tile of this workgroup
  uint32_t red32[kWaves];
  uint64_t red64[kWaves];
  uint32_t cls_cnt[kWaves][8];
  uint32_t ehist[24];      // rule P: values per scale offset e
  uint32_t words[256];     // binning pattern words of the current segment
  uint32_t bitmap[512];    // overlap check of a pattern (up to HIST_S_MAX sub-bins)
#ifdef HISTMI_TIMELINE
  uint32_t tl_n;           // timeline records written by this workgroup
#endif
};

// Per-workgroup timeline (diagnostic build only, -DHISTMI_TIMELINE: libhistmi_timeline.so).
// Thread 0 of each of the first kTlWgs workgroups records up to kTlPer events, each one
// word: phase << 56 | segment << 40 | the 100 MHz device clock (40 bits).  The recording
// adds one store per event and changes no step of the path; the default build compiles it
// out.  Phases: 0 entry, 2 segment set up (decision taken, table staged), 3 tile counted,
// 4 flushed (and, in multi-segment launches, the finalizer verdict known), 5 finalizer
// start, 6 merged, 7 finalizer done, 8 exit, 9 flush start (every wavefront's adds done),
// 10 table summed, 11 atomics issued, 12 sequencer lock taken, 13 batch decided (segment
// field: chunks), 14 lock released, 15 batch loaded (segment field: chunks present).
#ifdef HISTMI_TIMELINE
constexpr uint32_t kTlWgs = 2048, kTlPer = 256;
__device__ uint64_t g_timeline[kTlWgs * kTlPer];
#define TL(c_, ph_, seg_)                                                                              \
  do {                                                                                                 \
    if (threadIdx.x == 0) {                                                                            \
      const uint32_t i_ = (c_).tl_n++;                                                                 \
      if (i_ < kTlPer && blockIdx.x < kTlWgs)                                                          \
        g_timeline[blockIdx.x * kTlPer + i_] = ((uint64_t)(ph_) << 56) | ((uint64_t)((seg_) & 0xFFFF) << 40) | \
                                               ((uint64_t)wall_clock64() & ((1ull << 40) - 1));        \
    }                                                                                                  \
  } while (0)
#else
#define TL(c_, ph_, seg_) \
  do {                    \
  } while (0)
#endif

// ------------------------------------------------------------------ block helpers

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }
__device__ __forceinline__ uint32_t wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int o) {
  uint32_t lo = __shfl_xor((uint32_t)v, o, 64);
  uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
  return ((uint64_t)hi << 32) | lo;
}

__device__ uint32_t block_sum_u32(uint32_t v, Ctl &c) {
  v = wave_sum_u32(v);
  if (lane_id() == 0) c.red32[wave_id()] = v;
  __syncthreads();
  uint32_t s = 0;
#pragma unroll
  for (uint32_t w = 0; w < kWaves; ++w) s += c.red32[w];
  __syncthreads();
  return s;
}

// True iff p holds on every thread: one ballot per wavefront (no cross-lane traffic), the
// four results meet in LDS.
__device__ bool block_all(bool p, Ctl &c) {
  const uint64_t fails = __ballot(!p);
  if (lane_id() == 0) c.red32[wave_id()] = fails ? 1u : 0u;
  __syncthreads();
  uint32_t any = 0;
#pragma unroll
  for (uint32_t w = 0; w < kWaves; ++w) any |= c.red32[w];
  __syncthreads();
  return any == 0u;
}

__device__ uint64_t block_sum_u64(uint64_t v, Ctl &c) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += shfl_xor_u64(v, o);
  if (lane_id() == 0) c.red64[wave_id()] = v;
  __syncthreads();
  uint64_t s = 0;
#pragma unroll
  for (uint32_t w = 0; w < kWaves; ++w) s += c.red64[w];
  __syncthreads();
  return s;
}

__device__ uint64_t block_max_u64(uint64_t v, Ctl &c) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t u = shfl_xor_u64(v, o);
    v = u > v ? u : v;
  }
  if (lane_id() == 0) c.red64[wave_id()] = v;
  __syncthreads();
  uint64_t s = 0;
#pragma unroll
  for (uint32_t w = 0; w < kWaves; ++w) s = c.red64[w] > s ? c.red64[w] : s;
  __syncthreads();
  return s;
}

// Ordering of cross-workgroup communication.  Every location that workgroups share inside a
// launch (partial counts, tickets, decisions, stream state) is only touched through
// agent-scope atomics and agent-scope (sc1) loads and stores, which are performed at the
// device's coherence point.  What remains to order is a thread's earlier accesses before its
// later signal (a ticket or a flag): waiting until the earlier ones are acknowledged does
// that.  An agent-scope fence would also write back and invalidate the whole L2 of the XCD,
// which costs about a microsecond each and serialises the many flushes of a launch.
// Building with -DHISTMI_STRICT_FENCES uses those fences instead.
__device__ __forceinline__ void order_global() {
#ifdef HISTMI_STRICT_FENCES
  __threadfence();
#else
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#endif
}

// Device-memory pointer.  Pointers that the kernel loads from memory (the stream state's ring
// and trace arrays, a segment's buffers) reach it as generic pointers; a generic access is a
// FLAT instruction, which counts against both the vector-memory and the LDS counters and so
// makes every later wait a wait for all outstanding memory operations.  Every access below
// goes to device memory, never LDS, and says so.
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> gmem(T *p) {
  return (gptr<T>)p;
}

template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
  return __hip_atomic_load(gmem(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T *p, T v) {
  __hip_atomic_store(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded spin by thread 0 until the decision tag at p carries generation `gen`.  Returns
// the tag, or 0 after `polls` polls (counted in diag[1] and in the stream's wait_timeouts):
// the caller then runs the per-wavefront kernel, which needs no pattern, so a timeout costs
// speed and a trace entry, never counts.  (A chunk that gave up still writes its histogram
// into the stream's ring; the ring holds every chunk that two launches in flight can
// produce, so that write never lands on an entry the sequencer still needs.)
__device__ uint64_t spin_for_tag(const uint64_t *p, uint32_t gen, uint32_t polls, uint32_t *diag,
                                 uint64_t *st_timeouts) {
  for (uint32_t i = 0; i < polls; ++i) {
    const uint64_t tag = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tag_gen(tag) == gen) {
#ifdef HISTMI_STRICT_FENCES
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#endif
      return tag;
    }
    __builtin_amdgcn_s_sleep(8);
  }
  atomicAdd(&diag[1], 1u);
  __hip_atomic_fetch_add(st_timeouts, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return 0;
}

// ------------------------------------------------------------------ rule P on the device
//
// Pattern from a past histogram (the paper recomputes the indices from the past stream's
// histograms, Sec. III.B, without giving a rule).  Thread t holds h(t); N = sum h.
//   256*rmax <= S: every value gets rmax.  N == 0: every value gets 1.
//   Otherwise r_t(v) = min(rmax, pow2ceil(max(1, ceil(h(v) 2^t / N)))) at the largest t in
//   [0, min(24, clz64(N))] with sum_v r_t(v) <= S (the sum grows with t).
//   Values are laid out by (r descending, value ascending); bases are running sums.
//
// Evaluated without division and with one barrier for the search.  For h > 0 let e be the
// largest e >= 0 with h 2^e <= N.  Then ceil(h 2^t / N) <= 2^k holds iff k >= t - e, so
// log2 r_t(v) = min(log2 rmax, max(0, t - e(v))) (and 0 for h = 0).  The sum at scale t is
// therefore 256 + sum over e < t of n_e (2^min(log2 rmax, t - e) - 1), with n_e the number of
// values at e: a 24-bucket histogram of e in LDS gives every scale's sum, lane t of each
// wavefront evaluates scale t, and one ballot picks the largest that fits.

// e(v) as above: h 2^e has the bit length of N, or one less when that would exceed N.
__device__ __forceinline__ uint32_t rule_p_e(uint64_t h, uint64_t N) {
  if (h == 0) return 64u;
  const uint32_t bn = 64u - (uint32_t)__clzll((long long)N), bh = 64u - (uint32_t)__clzll((long long)h);
  uint32_t e = bn - bh;
  if ((h << e) > N) --e;   // bh + e = bn <= 64: no overflow; h <= N makes e >= 0 here
  return e;
}

// Returns this thread's pattern word; *kind_lg = the table kind (KIND_UNIFORM << 8 | log2 r
// when every value has the same r, which with this layout puts value v at v * r; else
// KIND_LOOKUP << 8).  All threads call.
__device__ uint32_t rule_p_word(uint64_t h, uint64_t N, uint32_t S, uint32_t rmax, Ctl &c, uint32_t *kind_lg) {
  const uint32_t t = threadIdx.x;
  const uint32_t rmax_lg = 31u - (uint32_t)__clz((int)rmax);
  const uint32_t lane = lane_id(), w = wave_id();
  uint32_t cls;
  if (256u * rmax <= S) {
    cls = rmax_lg;
  } else if (N == 0) {
    cls = 0;
  } else {
    const uint32_t T = min(24u, (uint32_t)__clzll((long long)N));
    const uint32_t e = rule_p_e(h, N);
    if (t < 24) c.ehist[t] = 0;
    __syncthreads();
    if (e < 24) atomicAdd(&c.ehist[e], 1u);
    __syncthreads();
    // lane l of every wavefront: the sum at scale l (the same in all four wavefronts)
    uint32_t sum = 256;
    for (uint32_t x = 0; x < lane && x < 24; ++x) {
      const uint32_t d = min(rmax_lg, lane - x);
      sum += c.ehist[x] * ((1u << d) - 1u);
    }
    const uint64_t fits = __ballot(lane <= T && sum <= S);   // a prefix 0..t* (scale 0 always fits)
    const uint32_t ts = 63u - (uint32_t)__clzll((long long)fits);
    cls = (e >= ts) ? 0u : min(rmax_lg, ts - e);
  }
  // layout by (r descending, value ascending)
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t rank = 0;
#pragma unroll
  for (uint32_t k = 0; k < 7; ++k) {
    const uint64_t m = __ballot(cls == k);
    if (lane == 0) c.cls_cnt[w][k] = (uint32_t)__popcll(m);
    if (cls == k) rank = (uint32_t)__popcll(m & below);
  }
  __syncthreads();
  for (uint32_t w2 = 0; w2 < w; ++w2) rank += c.cls_cnt[w2][cls];
  uint32_t offset = 0;
  for (uint32_t k = cls + 1; k < 7; ++k) {
    uint32_t cnt = 0;
    for (uint32_t w2 = 0; w2 < kWaves; ++w2) cnt += c.cls_cnt[w2][k];
    offset += cnt << k;
  }
  // one class holding all 256 values: the uniform table
  uint32_t same = 0;
  for (uint32_t w2 = 0; w2 < kWaves; ++w2) same += c.cls_cnt[w2][cls];
  *kind_lg = (same == 256u) ? (((uint32_t)KIND_UNIFORM << 8) | cls) : ((uint32_t)KIND_LOOKUP << 8);
  __syncthreads();
  return (offset + (rank << cls)) | (cls << 16);
}

// ------------------------------------------------------------------ table staging

__device__ __forceinline__ void zero_words(uint32_t *lds, uint32_t words) {
  u32x4 *p = reinterpret_cast<u32x4 *>(lds);
  const u32x4 z = {0u, 0u, 0u, 0u};
  for (uint32_t i = threadIdx.x; i < (words >> 2); i += kBlock) p[i] = z;
}

// Clear the counting table once per workgroup; from then on table_bin leaves it zero.  Ends
// with a barrier.
__device__ __forceinline__ void zero_table(uint32_t *lds, const Params &P) {
  zero_words(lds, P.table_words);
  __syncthreads();
}

// Check c.words as a pattern of S sub-bins and at most rmax per value; choose the kind.
// Returns KIND_UNIFORM (c.lg set) or KIND_LOOKUP for a valid pattern, KIND_WAVE otherwise.
__device__ uint32_t classify_pattern(Ctl &c, uint32_t S, uint32_t rmax, uint32_t S_cap, uint32_t rmax_cap,
                                     bool have_lookup) {
  const uint32_t t = threadIdx.x;
  const uint32_t w = c.words[t];
  const uint32_t base = w & 0xFFFFu, lg = (w >> 16) & 0xFFu, hi = w >> 24;
  const bool rmax_ok = rmax >= 1 && rmax <= rmax_cap && (rmax & (rmax - 1)) == 0 && S <= S_cap;
  bool ok = rmax_ok && hi == 0 && lg <= 6 && (1u << lg) <= rmax && base + (1u << lg) <= S;
  for (uint32_t i = t; i < 512; i += kBlock) c.bitmap[i] = 0;
  __syncthreads();
  if (ok) {
    const uint32_t lo_b = base, hi_b = base + (1u << lg);   // [lo_b, hi_b)
    for (uint32_t wi = lo_b >> 5; wi <= ((hi_b - 1) >> 5); ++wi) {
      const uint32_t s0 = wi << 5;
      const uint32_t a = lo_b > s0 ? lo_b - s0 : 0u;
      const uint32_t b = hi_b - s0 < 32u ? hi_b - s0 : 32u;
      const uint32_t mask = (b - a == 32u) ? 0xFFFFFFFFu : (((1u << (b - a)) - 1u) << a);
      const uint32_t old = atomicOr(&c.bitmap[wi], mask);
      if (old & mask) ok = false;
    }
  }
  if (!block_all(ok, c)) return KIND_WAVE;
  const uint32_t lg0 = (c.words[0] >> 16) & 0xFFu;
  const bool uni = (lg == lg0) && (base == (t << lg0));
  if (block_all(uni, c)) {
    c.lg = lg0;
    return KIND_UNIFORM;
  }
  return have_lookup ? KIND_LOOKUP : KIND_WAVE;
}

// KIND_LOOKUP: build the lane-replicated lookup table,
// look[v * RR + j] = byte address of sub-bin base(v) + (j mod r(v)), j = lane mod RR.
// (The counting table itself is already zero: see table_bin.)  Other kinds need nothing.
__device__ __forceinline__ void stage_table(uint32_t *lds, const Params &P, Ctl &c, uint32_t kind) {
  const uint32_t t = threadIdx.x;
  if (kind == KIND_LOOKUP) {
    const uint32_t w = c.words[t];
    const uint32_t base = w & 0xFFFFu, rmask = (1u << ((w >> 16) & 0xFFu)) - 1u;
    const uint32_t rr_lg = P.look_rr_lg, rr = 1u << rr_lg;
    uint32_t *look = lds + P.look_off + (t << rr_lg);
    const uint32_t tb = lds_addr_of(lds);
    for (uint32_t j = 0; j < rr; ++j) {
      const uint32_t jj = (j + t) & (rr - 1u);     // rotate so a wavefront's stores hit distinct banks
      look[jj] = tb + ((base + (jj & rmask)) << 2);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ the hot loop

template <int KIND>
struct Adder {
  uint32_t a;      // LDS byte address: KIND_WAVE: this wave's table; UNIFORM: table + (lane mod r) * 4;
                   // LOOKUP: this lane's column of the lookup table
  uint32_t s;      // UNIFORM: lg + 2; LOOKUP: log2(RR) + 2
  uint32_t lane;   // WAVE_AGG: this lane's index in the wavefront
  __device__ __forceinline__ void add(uint32_t v) const {
    uint32_t addr;
    if (KIND == KIND_WAVE_AGG) {
      // peel the first active lane's value: its holders add once, by their count
      const uint32_t v0 = __builtin_amdgcn_readfirstlane(v);
      const uint64_t eq = __ballot(v == v0);
      if (v != v0) {
        __hip_atomic_fetch_add((lu32 *)(uintptr_t)(a + (v << 2)), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      } else if (lane == (uint32_t)__builtin_ctzll(eq)) {
        __hip_atomic_fetch_add((lu32 *)(uintptr_t)(a + (v0 << 2)), (uint32_t)__popcll(eq), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      return;
    } else if (KIND == KIND_WAVE) {
      addr = a + (v << 2);
    } else if (KIND == KIND_UNIFORM) {
      addr = (v << s) + a;
    } else {
      addr = *(const lu32 *)(uintptr_t)((v << s) + a);   // absolute address of this lane's sub-bin
    }
    __hip_atomic_fetch_add((lu32 *)(uintptr_t)addr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __device__ __forceinline__ void add16(const u32x4 &x) const {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t d = x[q];
      add(d & 255u);
      add((d >> 8) & 255u);
      add((d >> 16) & 255u);
      add(d >> 24);
    }
  }
};

// U 16-byte vectors per lane (U x 1 KiB per wavefront): the unit of the load pipeline.  The
// loads of step q + 1 are issued before the bytes of step q go into the table, so every wave
// keeps U x 1 KiB of HBM reads outstanding while it works on the LDS.
template <int U>
struct Pipe {
  u32x4 cur[U];
  __device__ __forceinline__ void load(gu32x4 *v, uint64_t i, uint64_t stride) {
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = __builtin_nontemporal_load(v + i + u * stride);
  }
};

// A tile's bytes [a0, a0 + len) as the wide loads see them: nv 16-byte vectors from the
// aligned address b0, in nfull whole steps of U x 4 KiB (the workgroup starts at step r0 and
// wraps, so that workgroups working on equal-sized tiles at the same time do not all address
// the same HBM channels), then the remaining vectors; the unaligned head and tail (< 16
// bytes each) go through single-byte loads.  Only a0 and len are kept between priming and
// counting; the rest is recomputed (a few scalar operations) to save registers.
struct Range {
  uint64_t a0, len;
};
template <int U>
struct RangeLayout {
  static constexpr uint64_t step = (uint64_t)U * kBlock;
  uint64_t b0, nv, nfull, r0;
  __device__ __forceinline__ RangeLayout(const Range &r, uint32_t rot) {
    const uint64_t a1 = r.a0 + r.len;
    b0 = (r.a0 + 15u) & ~(uint64_t)15u;
    const uint64_t b1 = a1 & ~(uint64_t)15u;
    nv = b0 < b1 ? (b1 - b0) >> 4 : 0u;
    nfull = nv / step;
    r0 = nfull ? (uint64_t)rot % nfull : 0u;
  }
};

// Issue the tile's first step of loads.  The loads carry no table state, so a tile can be
// primed before the workgroup knows which table its segment will count into.
template <int U>
__device__ __forceinline__ Range prime_range(Pipe<U> &a, uint64_t a0, uint64_t len, uint32_t rot) {
  const Range r{a0, len};
  const RangeLayout<U> L(r, rot);
  if (L.nfull) a.load((gu32x4 *)L.b0, L.r0 * L.step + threadIdx.x, kBlock);
  return r;
}

// Count a primed tile.  mid() runs once, halfway through the tile's steps (at the start when
// the tile has fewer than two steps): it gives the workgroup's control thread a point at
// which earlier requests have long returned, to read them and issue follow-up loads.
template <int KIND, int U, typename Mid>
__device__ __forceinline__ void run_primed(const Adder<KIND> &ad, const Range &r, uint32_t rot, Pipe<U> &a,
                                           Mid &&mid) {
  const RangeLayout<U> L(r, rot);
  const uint64_t step = L.step;
  const uint32_t t = threadIdx.x;
  gu8 *pg = (gu8 *)r.a0;
  if (L.nfull < 2) mid();
  if (L.nv == 0) {
    for (uint64_t i = t; i < r.len; i += kBlock) ad.add(pg[i]);
    return;
  }
  const uint64_t b1 = L.b0 + (L.nv << 4), a1 = r.a0 + r.len;
  if (t < L.b0 - r.a0) ad.add(pg[t]);
  if (t < a1 - b1) ad.add(((gu8 *)b1)[t]);
  gu32x4 *v = (gu32x4 *)L.b0;
  if (L.nfull) {
    Pipe<U> b;
    const uint64_t half = L.nfull >> 1;
    for (uint64_t q = 0; q < L.nfull; ++q) {
      const bool more = q + 1 < L.nfull;
      if (more) {
        uint64_t s1 = q + 1 + L.r0;
        if (s1 >= L.nfull) s1 -= L.nfull;
        b.load(v, s1 * step + t, kBlock);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) ad.add16(a.cur[u]);
      if (more) a = b;
      if (q + 1 == half) mid();
    }
  }
  for (uint64_t i = L.nfull * step + t; i < L.nv; i += kBlock) ad.add16(__builtin_nontemporal_load(v + i));
}

// One buffer spread over the whole grid: workgroup g takes the 4 KiB blocks g, g + G,
// g + 2G, ... of the aligned middle, U blocks per step (next step prefetched); workgroup 0
// also takes the unaligned head and tail.  The counting table is cleared (zero_table, which
// ends with a barrier) while the first step's loads are in flight.
template <int KIND, int U>
__device__ void run_strided(uint32_t *lds, const Params &P, const Adder<KIND> &ad, const uint8_t *p, uint64_t len) {
  const uint32_t t = threadIdx.x, g = blockIdx.x, G = gridDim.x;
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(p), a1 = a0 + len;
  const uintptr_t b0 = (a0 + 15u) & ~static_cast<uintptr_t>(15u), b1 = a1 & ~static_cast<uintptr_t>(15u);
  gu8 *pg = (gu8 *)p;
  if (b0 >= b1) {
    zero_table(lds, P);
    if (g == 0)
      for (uint64_t i = t; i < len; i += kBlock) ad.add(pg[i]);
    return;
  }
  gu32x4 *v = (gu32x4 *)b0;
  const uint64_t nv = (b1 - b0) >> 4;
  const uint64_t stride = (uint64_t)G * kBlock;
  // block base of this workgroup's s-th full step: g*256 + s*U*stride; full iff its last
  // vector (lane 255 of block U-1) is inside
  uint64_t base = (uint64_t)g * kBlock;
  const uint64_t span = (uint64_t)(U - 1) * stride + (kBlock - 1);
  const bool full = base + span < nv;   // uniform over the workgroup
  Pipe<U> a, b;
  if (full) a.load(v, base + t, stride);
  zero_table(lds, P);
  if (g == 0) {
    if (t < b0 - a0) ad.add(pg[t]);
    if (t < a1 - b1) ad.add(((gu8 *)b1)[t]);
  }
  if (full) {
    for (;;) {
      const uint64_t nb = base + (uint64_t)U * stride;
      const bool more = nb + span < nv;
      if (more) b.load(v, nb + t, stride);
#pragma unroll
      for (int u = 0; u < U; ++u) ad.add16(a.cur[u]);
      base = nb;
      if (!more) break;
      a = b;
    }
  }
  for (uint64_t i = base + t; i < nv; i += stride) ad.add16(__builtin_nontemporal_load(v + i));
}

// Sum this thread's bin (value t) out of the table, clearing each sub-bin as it is read.
// Every sub-bin the adds can touch belongs to exactly one value, so after all threads have
// done this the whole counting table is zero again and the next segment needs no clearing
// pass (the table is cleared once when the workgroup starts).  A workgroup's last flush
// (CLEAR false) leaves the table as it is.
template <bool CLEAR = true>
__device__ uint32_t table_bin(uint32_t *lds, const Ctl &c, uint32_t kind, uint32_t lg) {
  const uint32_t t = threadIdx.x;
  uint32_t h = 0;
  if (kind == KIND_WAVE || kind == KIND_WAVE_AGG) {
#pragma unroll
    for (uint32_t w = 0; w < kWaves; ++w) {
      h += lds[(w << 8) | t];
      if (CLEAR) lds[(w << 8) | t] = 0u;
    }
  } else if (kind == KIND_UNIFORM && lg >= 4) {
    // value t's r sub-bins are one row of r / 4 16-byte quads: read four quads at a time
    // (one wait per four reads instead of one per word), then clear them.  The quad order is
    // rotated by row so that the lanes served together touch distinct banks, whether a
    // 16-byte access is served 8 lanes at a time over 32 banks or 16 lanes over 64: rows that
    // share a bank window get distinct rotations in every aligned group of 8 and of 16 lanes.
    const uint32_t nq = 1u << (lg - 2);
    const uint32_t rot = lg == 4 ? (t >> 1) + (t >> 3) : lg == 5 ? t + (t >> 3) : t;
    u32x4 *row = reinterpret_cast<u32x4 *>(lds + (t << lg));
    const u32x4 z = {0u, 0u, 0u, 0u};
    for (uint32_t k0 = 0; k0 < nq; k0 += 4) {
      u32x4 x[4];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) x[u] = row[(k0 + u + rot) & (nq - 1u)];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) {
        h += x[u][0] + x[u][1] + x[u][2] + x[u][3];
        if (CLEAR) row[(k0 + u + rot) & (nq - 1u)] = z;
      }
    }
  } else if (kind == KIND_UNIFORM) {
    const uint32_t r = 1u << lg;   // at most 8 sub-bins per value
    for (uint32_t j = 0; j < r; ++j) {
      const uint32_t i = (t << lg) | ((j + t) & (r - 1u));
      h += lds[i];
      if (CLEAR) lds[i] = 0u;
    }
  } else {
    // any pattern: eight reads in flight at a time, then clear
    const uint32_t w = c.words[t];
    const uint32_t base = w & 0xFFFFu, r = 1u << ((w >> 16) & 0xFFu);
    for (uint32_t j0 = 0; j0 < r; j0 += 8) {
      uint32_t x[8];
#pragma unroll
      for (uint32_t u = 0; u < 8; ++u) x[u] = (j0 + u < r) ? lds[base + j0 + u] : 0u;
#pragma unroll
      for (uint32_t u = 0; u < 8; ++u) {
        if (j0 + u < r) {
          h += x[u];
          if (CLEAR) lds[base + j0 + u] = 0u;
        }
      }
    }
  }
  return h;
}

// ------------------------------------------------------------------ segments

__device__ __forceinline__ SegDesc load_seg(const Params &P, uint32_t s) {
  return P.single ? P.seg0 : P.segs[s];
}

// Stage segment `sd`: pick the table kind (from the launch, or from the stream's decision)
// and prepare the LDS.  Returns the kind; sets c.lg / c.used_mode / c.words.
__device__ __forceinline__ uint32_t begin_segment(uint32_t *lds, const Params &P, Ctl &c, const SegDesc &sd,
                                                  uint64_t hint) {
  const uint32_t t = threadIdx.x;
  uint32_t kind;
  uint32_t S = P.pat_S;
  if (sd.chunk < 0) {
    kind = P.kind;
    if (kind == KIND_UNIFORM) c.lg = P.uni_lg;
    if (kind == KIND_LOOKUP) c.words[t] = P.pat_words[t];
    c.used_mode = (kind == KIND_WAVE) ? HIST_MODE_WAVEHIST : (kind == KIND_WAVE_AGG) ? HIST_MODE_WAVEAGG
                                                                                       : HIST_MODE_AHIST;
    __syncthreads();
  } else {
    StreamDev *st = P.st + sd.stream_idx;
    const int64_t k = (int64_t)P.chunk_base + sd.chunk;
    uint32_t dmode;
    if (sd.chunk == kServerChunk) {
      // served request: the stream's latest decision, whatever has been published (no wait)
      const Decision *d = &st->slots[0];
      if (t == 0) c.tag = ld_agent(&d->tag);
      __syncthreads();
      const uint64_t tag = c.tag;
      const uint32_t kind_lg = tag_kind_lg(tag);
      dmode = tag_gen(tag) == 0 ? (uint32_t)HIST_MODE_WAVEHIST : tag_mode(tag);
      const uint32_t mode = P.forced ? P.forced : dmode;
      if (mode == HIST_MODE_AHIST && tag_gen(tag) != 0 && (kind_lg >> 8) == KIND_UNIFORM &&
          (256u << (kind_lg & 0xFFu)) <= P.table_words) {
        // a uniform table is carried by the tag alone, which this library's own epilogue
        // stored in one piece: no pattern words to read or check
        if (t == 0) {
          c.lg = kind_lg & 0xFFu;
          c.used_mode = HIST_MODE_AHIST;
        }
        __syncthreads();
        return KIND_UNIFORM;
      }
      if (tag_gen(tag) == 0) {
        c.words[t] = t;
        S = 256;
      } else {
        // requests of one stream may finish together and overwrite each other's words: the
        // words are checked as a pattern below, and any mix that passes is a valid pattern
        c.words[t] = ld_agent(&d->words[t]);
        S = ld_agent(&d->S);
      }
    } else {
      // an ordered stream's decision was made by this library's own epilogue: thread 0 takes
      // its tag (one load, usually already done at the switch: see tag_prefetch), decides the
      // table from it and publishes the choice with one barrier; the pattern words are read
      // only when the lookup table or the trace needs them
      const int64_t j = k - 1 - (int64_t)P.lag;
      const bool traced = (uint64_t)k < P.trace_cap;
      const Decision *d = &P.slots[(uint64_t)(j >= 0 ? j : 0) % P.nslot];
      if (t == 0) {
        // no history, or (never expected) a wait that timed out: the per-wavefront kernel
        // with the identity pattern
        uint64_t tag = make_tag(0, HIST_MODE_WAVEHIST, (uint32_t)KIND_UNIFORM << 8);
        if (sd.known) {
          // the host knew this decision (it depends on the chunk sizes only): no wait
          tag = make_tag((sd.known & kKnownCold) ? 0u : 1u, (sd.known >> 16) & 0xFFu, sd.known & 0xFFFFu);
        } else if (j >= 0) {
          const uint32_t want = (uint32_t)(j + 1);
          const uint64_t got = (tag_gen(hint) == want)
                                   ? hint
                                   : spin_for_tag(&d->tag, want, P.wait_polls, P.diag,
                                                  &P.st[sd.stream_idx].wait_timeouts);
          if (got) tag = got;
        }
        const uint32_t mode = P.forced ? P.forced : tag_mode(tag);
        const uint32_t kind_lg = tag_kind_lg(tag);
        uint32_t kd, lg = 0;
        if (mode == HIST_MODE_AHIST) {
          kd = kind_lg >> 8;
          lg = kind_lg & 0xFFu;
          const uint32_t Sd = (kd == KIND_LOOKUP && tag_gen(tag) != 0) ? ld_agent(&d->S) : 256u;
          if ((kd == KIND_LOOKUP && (P.look_words == 0 || Sd > P.pat_S)) ||
              (kd == KIND_UNIFORM && (256u << lg) > P.table_words) || kd > KIND_LOOKUP) {
            kd = KIND_WAVE;   // no room for this pattern's tables (cannot happen with rule P)
            atomicAdd(&P.diag[0], 1u);
          }
        } else {
          kd = (mode == HIST_MODE_WAVEAGG) ? KIND_WAVE_AGG : KIND_WAVE;
        }
        if (traced)   // the earliest start of this chunk's counting, over its workgroups
          __hip_atomic_fetch_min(gmem(&P.time_trace[3u * (uint64_t)k]), (uint64_t)wall_clock64(), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        c.tag = tag;
        c.kind = kd;
        c.lg = lg;
        c.used_mode = (kd == KIND_WAVE) ? HIST_MODE_WAVEHIST : (kd == KIND_WAVE_AGG) ? HIST_MODE_WAVEAGG
                                                                                     : HIST_MODE_AHIST;
      }
      __syncthreads();
      kind = c.kind;
      // each thread writes and later reads only its own value's word (lookup staging, table
      // sums, trace), so no barrier is needed after this
      if (kind == KIND_LOOKUP || traced) {
        if (tag_gen(c.tag) == 0) {
          c.words[t] = t;
        } else if ((tag_kind_lg(c.tag) >> 8) == KIND_UNIFORM) {   // the words follow from the tag
          const uint32_t lg = tag_kind_lg(c.tag) & 0xFFu;
          c.words[t] = (t << lg) | (lg << 16);
        } else {
          c.words[t] = ld_agent(&d->words[t]);
        }
      }
      stage_table(lds, P, c, kind);
      return kind;
    }
    const uint32_t mode = P.forced ? P.forced : dmode;
    __syncthreads();
    if (mode == HIST_MODE_AHIST) {
      kind = classify_pattern(c, S, st->rmax, P.pat_S, HIST_RMAX_MAX, P.look_words != 0);
      if (kind == KIND_WAVE && t == 0) atomicAdd(&P.diag[0], 1u);
    } else if (mode == HIST_MODE_WAVEAGG) {
      kind = KIND_WAVE_AGG;
    } else {
      kind = KIND_WAVE;
    }
    if (t == 0)
      c.used_mode = (kind == KIND_WAVE) ? HIST_MODE_WAVEHIST : (kind == KIND_WAVE_AGG) ? HIST_MODE_WAVEAGG
                                                                                       : HIST_MODE_AHIST;
    __syncthreads();
  }
  stage_table(lds, P, c, kind);
  return kind;
}

// Epilogue of a served request (thread t holds bin t of its histogram h): the stream's
// running histogram grows by h (atomically: requests of one stream may finish in any order)
// and the stream's decision is recomputed from h alone (a window of one request).  Concurrent
// requests of one stream may overwrite each other's decision; any mix of words that passes
// the device check is still a valid pattern, so counts stay exact.
__device__ __forceinline__ void server_epilogue(const Params &P, Ctl &c, uint32_t sidx, uint32_t h) {
  const uint32_t t = threadIdx.x;
  StreamDev *st = P.st + sidx;
  atomicAdd(reinterpret_cast<unsigned long long *>(&st->acc[t]), (unsigned long long)h);
  st_agent(&st->mw[t], (uint64_t)h);
  const uint64_t N = block_sum_u64(h, c);
  const uint64_t mx = block_max_u64(h, c);
  const uint32_t mode = (100ull * mx > (uint64_t)st->theta * N) ? HIST_MODE_AHIST : HIST_MODE_WAVEHIST;
  uint32_t kind_lg;
  const uint32_t word = rule_p_word(h, N, st->S, st->rmax, c, &kind_lg);
  Decision *d = &st->slots[0];
  st_agent(&d->words[t], word);
  if (t == 0) {
    st_agent(&d->S, st->S);
    st_agent(&d->rmax, st->rmax);
  }
  order_global();
  __syncthreads();
  if (t == 0) st_agent(&d->tag, make_tag(1, mode, kind_lg));   // generation 1: "a decision exists"
}

// Rule P (Sec. III.B) for a window mw of N bytes (thread t holds bin t; all threads call):
// the pattern word for value t, and the table kind in *kind_lg.  When the budget S holds rmax
// sub-bins for every value, rule P gives every value rmax whatever the window: the pattern
// is the uniform table v * rmax and no block-wide pass is needed.
__device__ __forceinline__ uint32_t decide_pattern(const Params &P, Ctl &c, uint64_t mw, uint64_t N,
                                                   uint32_t *kind_lg) {
  const uint32_t t = threadIdx.x;
  if (256u * P.rmax <= P.S) {
    const uint32_t lg = (uint32_t)__builtin_ctz(P.rmax);
    *kind_lg = ((uint32_t)KIND_UNIFORM << 8) | lg;
    return (t << lg) | (lg << 16);
  }
  return rule_p_word(mw, N, P.S, P.rmax, c, kind_lg);
}

// Publish the decision made after chunk j into slot d (all threads call).  The chunk that
// runs with it (j + 1 + lag) reads the pattern words only for a lookup table; a uniform
// table's words follow from the tag (value v at v << lg), also for the chunk's trace, so the
// tag alone carries the decision and is stored at once, with nothing to wait for.  When the
// words are needed they are stored and acknowledged before the tag.
__device__ __forceinline__ void publish_decision(const Params &P, Decision *d, uint64_t j, uint32_t mode,
                                                 uint32_t kind_lg, uint32_t word) {
  const uint32_t t = threadIdx.x;
  const uint64_t tag = make_tag(j + 1, mode, kind_lg);
  const bool words_needed = (kind_lg >> 8) == KIND_LOOKUP;
  if (!words_needed) {
    if (t == 0) st_agent(&d->tag, tag);
    return;
  }
  st_agent(&d->words[t], word);
  if (t == 0) {
    st_agent(&d->S, P.S);
    st_agent(&d->rmax, P.rmax);
  }
  order_global();
  __syncthreads();
  if (t == 0) st_agent(&d->tag, tag);
}

// Sequencing of a stream with a moving window of W > 1 chunks.  MW_j needs the chunks in
// order, but chunks finish in any order; rather than have each chunk's finalizer wait for the
// one before it, every finalizer leaves its histogram (and size) in the ring and tries (one
// CAS) to become the stream's sequencer.  The sequencer keeps the window and its byte count in
// registers and takes the chunks in order for as long as the next one's histogram is there:
// MW += h_j - h_{j-W}, N += n_j - n_{j-W}, then the decision after chunk j.  Before it leaves
// it stores the window, releases the lock and looks once more, so a histogram that arrived
// while it held the lock is never left behind (its own finalizer's CAS failed only while the
// lock was held).  Nothing waits.
//
// The sequencer works in batches of B chunks, one memory round trip each: the ring entries
// of chunks j .. j + B - 1 (and of the chunks leaving the window) are loaded together;
// every entry carries its chunk's generation, so each wavefront finds with one ballot per
// chunk which of them are there, and which windows have a bin above theta percent of their
// bytes (Sec. III.C); the four wavefronts' results meet in LDS behind one barrier.  The
// chunks that are there, in order from j, are then decided and published.  An entry of a
// chunk leaving the window that is itself in the batch may not have been loaded yet; the
// chunk that needs it then counts as absent and is taken by the next batch.
// Batch sizes: as many chunks as fit beside the tile loop's registers (occupancy 4); the
// 128-bit arithmetic of change detection and of the collision criterion leaves room for fewer.
constexpr uint32_t kSeqBatch = 6;
constexpr uint32_t kSeqBatchExtra = 3;
constexpr uint32_t kWalkBatch = 8;   // walk_kernel: registers are no concern there, no collision sums
static_assert(kSeqBatch <= 8 && kSeqBatchExtra <= 4 && kWalkBatch <= 8, "per-chunk flags: bits 0-7 absent, 16-23 over theta, "
                                                    "24-31 alarms; collision sums for 4 chunks");

// Change detection for value t (Sec. III.B; the measure is our reading): its share of the
// window departs from its share of the Accumulator by more than pct percentage points,
// 100 * |mw * N_acc - acc * N_mw| > lim with lim = pct * N_mw * N_acc, exactly (never with an
// empty window or Accumulator).  The integers go up to 2^128, held as (hi, lo) 64-bit halves;
// their products take the GPU's quarter-rate 32-bit multiplies (about half a microsecond a
// chunk for the sequencer).  The walk_kernel launch, which has registers to spare (the
// counting kernel has not), first takes the test in double precision (share_departs_filtered).  Below 2^53
// every operand converts exactly, each of the two products and their difference is rounded
// once (relative 2^-53), and so is 100 x that; the limit is pct x a rounded product of two
// exact values.  The double comparison is therefore off by at most about 2^-51 of
// 100 (mw N_acc + acc N_mw) + lim.  It decides when it clears the limit by 2^-49 of that, either
// way.  Within that band (ties included), and for operands of 2^53 or more, the exact 128-bit
// test decides.
struct U128 {
  uint64_t hi, lo;
};
__device__ __forceinline__ U128 mul_64x64(uint64_t a, uint64_t b) { return {__umul64hi(a, b), a * b}; }
__device__ __forceinline__ bool gt_128(U128 a, U128 b) { return a.hi > b.hi || (a.hi == b.hi && a.lo > b.lo); }
__device__ __forceinline__ U128 sub_128(U128 a, U128 b) {
  return {a.hi - b.hi - (a.lo < b.lo ? 1u : 0u), a.lo - b.lo};
}
// pct * nmw * nacc (nmw, nacc < 2^64, pct <= 100; exact while the product is below 2^128)
__device__ __forceinline__ U128 alarm_limit(uint32_t pct, uint64_t nmw, uint64_t nacc) {
  const U128 p = mul_64x64(nmw, nacc);
  return {p.hi * pct + __umul64hi(p.lo, pct), p.lo * pct};
}
__device__ __forceinline__ bool share_departs(uint64_t mwv, uint64_t accv, uint64_t nmw, uint64_t nacc, U128 lim) {
  if (nmw == 0 || nacc == 0) return false;
  const U128 x = mul_64x64(mwv, nacc), y = mul_64x64(accv, nmw);
  const U128 d = gt_128(x, y) ? sub_128(x, y) : sub_128(y, x);
  const U128 d100 = {d.hi * 100u + __umul64hi(d.lo, 100u), d.lo * 100u};
  return gt_128(d100, lim);
}
__device__ __forceinline__ bool share_departs_filtered(uint64_t mwv, uint64_t accv, uint64_t nmw, uint64_t nacc,
                                                       uint32_t pct) {
  if (nmw == 0 || nacc == 0) return false;
  if (((mwv | accv | nmw | nacc) >> 53) == 0) {
    const double a = (double)mwv * (double)nacc, b = (double)accv * (double)nmw;
    const double d = 100.0 * __builtin_fabs(a - b);
    const double l = (double)pct * ((double)nmw * (double)nacc);
    const double e = 0x1p-49 * (100.0 * (a + b) + l);
    if (d > l + e) return true;
    if (d < l - e) return false;
  }
  return share_departs(mwv, accv, nmw, nacc, alarm_limit(pct, nmw, nacc));
}

// The alternative switching criterion (the paper leaves others to future work; our reading):
// the window's collision index sum_v p_v^2 above kappa percent, i.e.
// 100 * sum_v MW(v)^2 > kappa * N^2, in exact integers.  Each thread splits MW(t)^2 (a 128-bit
// value; MW(t) < 2^56) into limbs of bits [0,32), [32,64) and [64,128); 256 of each limb sum in
// 64 bits, and the sums give sum_v MW(v)^2 back.
__device__ __forceinline__ void square_limbs(uint64_t x, uint64_t *l) {
  const uint64_t lo = x * x;
  l[0] = lo & 0xFFFFFFFFu;
  l[1] = lo >> 32;
  l[2] = __umul64hi(x, x);
}
__device__ __forceinline__ U128 from_limbs(uint64_t s0, uint64_t s1, uint64_t s2) {
  const uint64_t lo = s0 + (s1 << 32);
  return {s2 + (s1 >> 32) + (lo < s0 ? 1u : 0u), lo};
}
__device__ __forceinline__ bool collision_above(U128 sq, uint64_t n, uint32_t kappa) {
  if (n == 0) return false;
  const U128 s100 = {sq.hi * 100u + __umul64hi(sq.lo, 100u), sq.lo * 100u};
  const U128 nn = mul_64x64(n, n);
  const U128 lim = {nn.hi * kappa + __umul64hi(nn.lo, kappa), nn.lo * kappa};
  return gt_128(s100, lim);
}
// The switch (Sec. III.C and the alternative): AHist iff the chosen test fires.
__device__ __forceinline__ uint32_t switch_mode(uint32_t criterion, bool maxbin, bool collision) {
  const bool ahist = criterion == HIST_CRIT_MAXBIN ? maxbin
                     : criterion == HIST_CRIT_COLLISION ? collision : (maxbin || collision);
  return ahist ? HIST_MODE_AHIST : HIST_MODE_WAVEHIST;
}

__device__ __forceinline__ uint64_t lane_u64(uint64_t v, uint32_t lane) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

template <uint32_t B, bool EXTRA, bool WALK = false>
__device__ __forceinline__ void sequence_stream(const Params &P, Ctl &c, StreamDev *st, uint64_t stop = ~0ull) {
  const uint32_t t = threadIdx.x, lane = lane_id();
  const uint32_t W = P.W, R = P.R, nslot = P.nslot;
  const uint32_t apct = P.alarm_pct;
  // EXTRA: the instantiation that can also run change detection and the collision criterion.
  // WALK: the walk_kernel launch of a stream whose decisions the host knows (uniform switch):
  // the decision after chunk j is AHist iff the window holds a byte, whatever the criterion,
  // so no collision sums are kept; the next batch's entries are loaded while this one is
  // decided, and the alarm test is filtered in double precision.  The walk ends at chunk
  // `stop` (the end of its launch's chunks) with no last look: the next launch's walk takes
  // over from there.
  const bool alarm_on = EXTRA && apct != 0;
  const bool coll_on = EXTRA && !WALK && P.criterion != HIST_CRIT_MAXBIN;
  uint32_t cb = 0;   // collision limb sums: this batch's buffer (three, so they clear without a barrier)
  const uint64_t *ring = st->ring;
  const uint64_t *ring_n = st->ring_n;
  uint8_t *alarm_trace = st->alarm_trace;
  Decision *slots = P.slots;
  auto wrap = [R](uint32_t s, uint32_t d) -> uint32_t { return s + d >= R ? s + d - R : s + d; };
  uint32_t par = 0;
  for (;;) {
    if (t == 0) {
      c.flag = (atomicCAS(&st->seq_lock, 0u, 1u) == 0u) ? 1u : 0u;
      if (coll_on && c.flag)
        for (uint32_t i = 0; i < 3 * 4 * 3; ++i) (&c.coll[0][0][0])[i] = 0;
    }
    __syncthreads();
    const bool holder = c.flag != 0;
    __syncthreads();
    if (!holder) return;
    TL(c, 12, 0);
    // the previous holder stored these before it released the lock (values every thread
    // shares are moved to scalar registers)
    uint64_t j = lane_u64(ld_agent(&st->done), 0);
    uint64_t N = lane_u64(ld_agent(&st->win_n), 0);
    uint64_t mw = ld_agent(&st->mw[t]);
    // change detection: the Accumulator in chunk order and its bytes
    uint64_t sacc = 0, NA = 0;
    if (alarm_on) {
      sacc = ld_agent(&st->sacc[t]);
      NA = lane_u64(ld_agent(&st->sacc_n), 0);
      if (t == 0) {   // kept in LDS while the lock is held
        c.alarms[0] = ld_agent(&st->alarms);
        c.alarms[1] = ld_agent(&st->first_alarm);
        c.alarms[2] = ld_agent(&st->last_alarm);
      }
    }
    // ring slots of chunk j and of chunk j - W (meaningful once j >= W), decision slot of j
    uint32_t sj = (uint32_t)(j % R);
    uint32_t so = sj >= W ? sj - W : sj + R - W;
    uint32_t dj = (uint32_t)(j % nslot);
    // change detection: a batch's alarms (this wavefront's ballots) travel with the next
    // batch's flags, so they cost no barrier of their own; thread 0 then records them
    uint32_t pend = 0, pcnt = 0;
    uint64_t pj = 0;
    auto record = [&](uint32_t al, uint64_t j0, uint32_t n) {
      if (t != 0) return;
      for (uint32_t b = 0; b < n; ++b) {
        const uint64_t q = j0 + b;
        const uint32_t hit = (al >> b) & 1u;
        if (hit) {
          ++c.alarms[0];
          if (c.alarms[1] == 0) c.alarms[1] = q + 1;
          c.alarms[2] = q + 1;
        }
        if (q < P.trace_cap) *gmem(&alarm_trace[q]) = (uint8_t)hit;
      }
    };
    // WALK: the next batch's entries, loaded while this one is decided (valid when `ahead`)
    uint64_t ne[WALK ? B : 1], neo[WALK ? B : 1], nnv = 0, nnov = 0;
    bool ahead = false;
    for (;;) {
      // one round trip: this thread's bins of chunks j + b and j + b - W, and in lane b the
      // sizes of those two chunks
      const uint32_t bl = lane < B ? lane : 0u;
      uint64_t e[B], eo[B], nv, nov;
      if (WALK && ahead) {
#pragma unroll
        for (uint32_t b = 0; b < B; ++b) {
          e[b] = ne[WALK ? b : 0];
          eo[b] = neo[WALK ? b : 0];
        }
        nv = nnv;
        nov = nnov;
      } else {
#pragma unroll
        for (uint32_t b = 0; b < B; ++b) {
          e[b] = ld_agent(&ring[(size_t)wrap(sj, b) * 256u + t]);
          eo[b] = ld_agent(&ring[(size_t)wrap(so, b) * 256u + t]);
        }
        nv = ld_agent(&ring_n[wrap(sj, bl)]);
        nov = ld_agent(&ring_n[wrap(so, bl)]);
      }
      if (WALK) {
        // chunks j + B .. j + 2B - 1, as they are now: one that is not complete yet reads as
        // absent, which ends this walk early (its last look then finds it)
        const uint32_t sj2 = wrap(sj, B), so2 = wrap(so, B);
#pragma unroll
        for (uint32_t b = 0; b < B; ++b) {
          ne[WALK ? b : 0] = ld_agent(&ring[(size_t)wrap(sj2, b) * 256u + t]);
          neo[WALK ? b : 0] = ld_agent(&ring[(size_t)wrap(so2, b) * 256u + t]);
        }
        nnv = ld_agent(&ring_n[wrap(sj2, bl)]);
        nnov = ld_agent(&ring_n[wrap(so2, bl)]);
        ahead = true;
      }
      uint32_t bad = 0, hot = 0;
      uint64_t m = mw, NN = N;
#pragma unroll
      for (uint32_t b = 0; b < B; ++b) {
        const uint64_t q = j + b;
        const uint32_t g = (uint32_t)(q + 1), go = (uint32_t)(q + 1 - W);
        const bool old = q >= W;
        const uint64_t n = lane_u64(nv, b), no = lane_u64(nov, b);
        bool ok = (uint32_t)(e[b] >> 32) == g && (uint32_t)(n >> kSizeBits) == (g & kSizeGenMask);
        if (old)
          ok = ok && (uint32_t)(eo[b] >> 32) == go && (uint32_t)(no >> kSizeBits) == (go & kSizeGenMask);
        m += (uint64_t)(uint32_t)e[b] - (old ? (uint64_t)(uint32_t)eo[b] : 0u);
        NN += (n & kSizeMask) - (old ? (no & kSizeMask) : 0u);
        if (__ballot(!ok) != 0) bad |= 1u << b;
        if (__ballot(100ull * m > (uint64_t)P.theta * NN) != 0) hot |= 1u << b;
        if (coll_on) {
          uint64_t l[3];
          square_limbs(m, l);
#pragma unroll
          for (uint32_t i = 0; i < 3; ++i)
            atomicAdd(reinterpret_cast<unsigned long long *>(&c.coll[cb][b][i]), (unsigned long long)l[i]);
        }
      }
      uint32_t *f = c.sflag[par];
      par ^= 1u;
      if (lane == 0) f[wave_id()] = bad | (hot << 16) | (alarm_on ? pend << 24 : 0u);
      __syncthreads();
      uint32_t fl = 0;
#pragma unroll
      for (uint32_t w = 0; w < kWaves; ++w) fl |= f[w];
      if (alarm_on && pcnt) record(fl >> 24, pj, pcnt);
      // the buffer of the batch before this one: every thread read it before this barrier
      const uint32_t cprev = cb == 0 ? 2u : cb - 1u;
      if (coll_on && t == 0)
        for (uint32_t i = 0; i < 4 * 3; ++i) (&c.coll[cprev][0][0])[i] = 0;
      // chunks j .. j + cnt - 1 are there (all four wavefronts saw every entry)
      uint32_t cnt = (uint32_t)__builtin_ctz((fl & 0xFFu) | (1u << B));
      if (WALK) cnt = j >= stop ? 0u : (stop - j < cnt ? (uint32_t)(stop - j) : cnt);
      TL(c, 15, cnt);
      uint32_t alarm = 0;
      // A batch whose decisions are all the uniform table (the budget holds rmax sub-bins for
      // every value), with no change detection and no collision criterion, differs from chunk to chunk only in the mode, which the hot flags carry: the window
      // moves by cnt chunks and thread 0 stores cnt tags in a short loop.  The general path
      // below decides chunk by chunk in unrolled code that runs from a cold instruction cache
      // (about 0.25 us a chunk, as much as the batch's load round trip for six chunks).
      if (!EXTRA && 256u * P.rmax <= P.S) {
#pragma unroll
        for (uint32_t b = 0; b < B; ++b)
          if (b < cnt) mw += (uint64_t)(uint32_t)e[b] - (j + b >= W ? (uint64_t)(uint32_t)eo[b] : 0u);
#pragma unroll 1
        for (uint32_t b = 0; b < cnt; ++b)
          N += (lane_u64(nv, b) & kSizeMask) - (j + b >= W ? (lane_u64(nov, b) & kSizeMask) : 0u);
        if (t == 0) {
          const uint32_t kind_lg = ((uint32_t)KIND_UNIFORM << 8) | (uint32_t)__builtin_ctz(P.rmax);
#pragma unroll 1
          for (uint32_t b = 0; b < cnt; ++b) {
            const uint32_t mode = ((fl >> (16 + b)) & 1u) ? (uint32_t)HIST_MODE_AHIST : (uint32_t)HIST_MODE_WAVEHIST;
            const uint32_t d = dj + b >= nslot ? dj + b - nslot : dj + b;
            st_agent(&slots[d].tag, make_tag(j + b + 1, mode, kind_lg));
          }
        }
      } else if (WALK) {
        // The walk after a push (decisions from the host, alarms on): every running sum of
        // the batch first (cheap adds), then the alarm tests, which do not depend on one
        // another.  With one wavefront per SIMD, a test per step would wait out its own
        // latency before the next could start.
        uint64_t wm[B], wa[B], wn[B], wna[B];
        {
          uint64_t m = mw, a = sacc, n = N, na = NA;
#pragma unroll
          for (uint32_t b = 0; b < B; ++b) {
            const bool old = j + b >= W;
            const uint64_t nb = lane_u64(nv, b) & kSizeMask;
            m += (uint64_t)(uint32_t)e[b] - (old ? (uint64_t)(uint32_t)eo[b] : 0u);
            n += nb - (old ? (lane_u64(nov, b) & kSizeMask) : 0u);
            a += (uint32_t)e[b];
            na += nb;
            wm[b] = m;
            wa[b] = a;
            wn[b] = n;
            wna[b] = na;
          }
        }
#pragma unroll
        for (uint32_t b = 0; b < B; ++b) {
          const bool dep = b < cnt && share_departs_filtered(wm[b], wa[b], wn[b], wna[b], apct);
          if (__ballot(dep) != 0) alarm |= 1u << b;
        }
        const uint32_t kind_lg = ((uint32_t)KIND_UNIFORM << 8) | (uint32_t)__builtin_ctz(P.rmax);
#pragma unroll
        for (uint32_t b = 0; b < B; ++b)
          if (b < cnt) {
            mw = wm[b];
            sacc = wa[b];
            N = wn[b];
            NA = wna[b];
            if (t == 0) {
              const uint32_t d = dj + b >= nslot ? dj + b - nslot : dj + b;
              const uint32_t mode = wn[b] > 0 ? (uint32_t)HIST_MODE_AHIST : (uint32_t)HIST_MODE_WAVEHIST;
              st_agent(&slots[d].tag, make_tag(j + b + 1, mode, kind_lg));
            }
          }
      } else {
      // the batch's decisions: a lookup pattern's words are stored as each is decided, and
      // the tags all go out at the end, after one fence for the whole batch (a tag may be
      // read only once its words are visible; a fence and a barrier per chunk cost more)
      bool words = false;
#pragma unroll
      for (uint32_t b = 0; b < B; ++b) {
        if (b >= cnt) break;
        const uint64_t q = j + b;
        const bool old = q >= W;
        mw += (uint64_t)(uint32_t)e[b] - (old ? (uint64_t)(uint32_t)eo[b] : 0u);
        N += (lane_u64(nv, b) & kSizeMask) - (old ? (lane_u64(nov, b) & kSizeMask) : 0u);
        uint32_t kind_lg;
        const uint32_t word = decide_pattern(P, c, mw, N, &kind_lg);
        bool coll = false;
        if (coll_on)
          coll = collision_above(from_limbs(c.coll[cb][b][0], c.coll[cb][b][1], c.coll[cb][b][2]), N, P.kappa);
        const uint32_t mode = WALK ? (N > 0 ? (uint32_t)HIST_MODE_AHIST : (uint32_t)HIST_MODE_WAVEHIST)
                                   : switch_mode(P.criterion, ((fl >> (16 + b)) & 1u) != 0, coll);
        const uint32_t d = dj + b >= nslot ? dj + b - nslot : dj + b;
        if ((kind_lg >> 8) == KIND_LOOKUP) {
          st_agent(&slots[d].words[t], word);
          if (t == 0) {
            st_agent(&slots[d].S, P.S);
            st_agent(&slots[d].rmax, P.rmax);
          }
          words = true;
        }
        if (t == 0) c.ptag[b] = make_tag(q + 1, mode, kind_lg);
        if (alarm_on) {
          sacc += (uint32_t)e[b];
          NA += lane_u64(nv, b) & kSizeMask;
          const bool dep = WALK ? share_departs_filtered(mw, sacc, N, NA, apct)
                                : share_departs(mw, sacc, N, NA, alarm_limit(apct, N, NA));
          if (__ballot(dep) != 0) alarm |= 1u << b;
        }
      }
      if (words) {                 // (the same in every thread: the kind is the workgroup's)
        order_global();            // this thread's words before any tag
        __syncthreads();           // every thread's, before thread 0 stores the tags
      }
      if (t == 0)
        for (uint32_t b = 0; b < cnt; ++b) {
          const uint32_t d = dj + b >= nslot ? dj + b - nslot : dj + b;
          st_agent(&slots[d].tag, c.ptag[b]);
        }
      }
      cb = cb == 2 ? 0u : cb + 1u;
      pend = alarm;
      pcnt = cnt;
      pj = j;
      j += cnt;
      sj = wrap(sj, cnt);
      so = wrap(so, cnt);
      dj = dj + cnt >= nslot ? dj + cnt - nslot : dj + cnt;
      TL(c, 13, cnt);
      if (cnt < B) break;
    }
    if (alarm_on && pcnt) {
      // the last batch's alarms
      uint32_t *fa = c.sflag[par];
      par ^= 1u;
      if (lane == 0) fa[wave_id()] = pend;
      __syncthreads();
      uint32_t al = 0;
#pragma unroll
      for (uint32_t w = 0; w < kWaves; ++w) al |= fa[w];
      record(al, pj, pcnt);
    }
    st_agent(&st->mw[t], mw);
    if (t == 0) {
      st_agent(&st->done, j);
      st_agent(&st->win_n, N);
    }
    if (alarm_on) {
      st_agent(&st->sacc[t], sacc);
      if (t == 0) {
        st_agent(&st->sacc_n, NA);
        st_agent(&st->alarms, c.alarms[0]);
        st_agent(&st->first_alarm, c.alarms[1]);
        st_agent(&st->last_alarm, c.alarms[2]);
      }
    }
    order_global();
    __syncthreads();
    if (t == 0) st_agent(&st->seq_lock, 0u);
    TL(c, 14, 0);
    if (WALK && j >= stop) return;
    order_global();
    // look once more: a chunk that arrived while the lock was held
    const uint64_t e = ld_agent(&ring[(size_t)sj * 256u + t]);
    const uint64_t n = ld_agent(&ring_n[sj]);
    const uint32_t g = (uint32_t)(j + 1);
    if (!block_all((uint32_t)(e >> 32) == g && (uint32_t)(n >> kSizeBits) == (g & kSizeGenMask), c)) return;
  }
}

// Rate of the shader's cycle counter in ticks per microsecond between two readings of it
// (s0, s1) and of the constant 100 MHz clock (w0, w1) taken in one workgroup.
__device__ __forceinline__ uint64_t clock_mhz(uint64_t s0, uint64_t w0, uint64_t s1, uint64_t w1) {
  return w1 > w0 ? (s1 - s0) * 100u / (w1 - w0) : 0u;
}

// Stream epilogue for chunk k of `bytes` bytes with histogram h (thread t holds bin t):
// Accumulator, the trace of what chunk k ran with, then the moving window, degeneracy switch
// and rule P (Sec. III.B, Sec. III.C).  With a window of one chunk (W = 1) the decision after
// chunk k depends on h_k alone, so epilogues of different chunks run independently; with
// W > 1, or with change detection (which needs the Accumulator in chunk order), the chunks
// are sequenced (see sequence_stream) -- unless the host knew every decision of the launch.
// Then no chunk of the launch waits for the walk.  Without change detection (`known` carries
// kUnwalked) the decision after chunk k depends only on which chunks of the window hold
// bytes, which the host passes in, and the window itself is rebuilt from the ring when it is
// next read.  With change detection (kWalkAfter) the chunk only leaves its entry in the ring,
// and a one-workgroup walk_kernel launch after the counting launch walks the chunks in order.
__device__ __forceinline__ void stream_epilogue(const Params &P, Ctl &c, uint32_t sidx, int64_t k, uint32_t h,
                                                uint64_t bytes, uint32_t known) {
  const uint32_t t = threadIdx.x;
  StreamDev *st = P.st + sidx;
  const bool traced = (uint64_t)k < P.trace_cap;
  // the shader's cycle counter and the constant-rate clock, read twice within this
  // workgroup: their ratio follows the engine clock while the epilogue ran (traced chunks)
  const uint64_t sclk0 = traced ? (uint64_t)clock64() : 0, wall0 = traced ? (uint64_t)wall_clock64() : 0;
  __hip_atomic_fetch_add(gmem(&st->acc[t]), (uint64_t)h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (traced) {
    st_agent(&st->pat_trace[(size_t)k * 256u + t], c.words[t]);
    if (t == 0) *gmem(&st->mode_trace[k]) = (uint8_t)c.used_mode;
  }
  if (P.W == 1 && P.alarm_pct == 0) {
    // degeneracy of the window (this chunk): AHist iff some bin exceeds theta percent (strict)
    const bool hot = 100ull * h > (uint64_t)P.theta * bytes;
    const bool maxbin = !block_all(!hot, c);
    bool coll = false;
    if (P.criterion != HIST_CRIT_MAXBIN) {
      // collision criterion: the limb sums of sum h^2 through LDS atomics
      if (t < 3) c.coll[0][0][t] = 0;
      __syncthreads();
      uint64_t l[3];
      square_limbs(h, l);
#pragma unroll
      for (uint32_t i = 0; i < 3; ++i)
        atomicAdd(reinterpret_cast<unsigned long long *>(&c.coll[0][0][i]), (unsigned long long)l[i]);
      __syncthreads();
      coll = collision_above(from_limbs(c.coll[0][0][0], c.coll[0][0][1], c.coll[0][0][2]), bytes, P.kappa);
      __syncthreads();
    }
    const uint32_t mode = switch_mode(P.criterion, maxbin, coll);
    uint32_t kind_lg;
    const uint32_t word = decide_pattern(P, c, h, bytes, &kind_lg);
    Decision *d = &P.slots[(uint64_t)k % P.nslot];
    st_agent(&d->hist[t], h);
    // the time the decision is ready, taken before it is published: a chunk that waits for
    // it begins counting later than this
    const uint64_t ready = wall_clock64();
    publish_decision(P, d, (uint64_t)k, mode, kind_lg, word);
    if (t == 0) {
      __hip_atomic_fetch_add(&st->done, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (traced) {
        st_agent(&P.time_trace[3u * (uint64_t)k + 1u], ready);
        st_agent(&P.time_trace[3u * (uint64_t)k + 2u], clock_mhz(sclk0, wall0, (uint64_t)clock64(), ready));
      }
    }
    return;
  }
  const uint32_t slot = (uint32_t)((uint64_t)k % P.R);
  st_agent(&st->ring[(size_t)slot * 256u + t], ((uint64_t)(uint32_t)(k + 1) << 32) | h);
  if (t == 0) {
    st_agent(&st->ring_n[slot], ((uint64_t)((uint32_t)(k + 1) & kSizeGenMask) << kSizeBits) | bytes);
    if (traced) {
      const uint64_t w = wall_clock64();
      st_agent(&P.time_trace[3u * (uint64_t)k + 1u], w);
      st_agent(&P.time_trace[3u * (uint64_t)k + 2u], clock_mhz(sclk0, wall0, (uint64_t)clock64(), w));
    }
  }
  if (known & kUnwalked) {
    if (t == 0) {
      const uint32_t mode = (known & kAfterAhist) ? HIST_MODE_AHIST : HIST_MODE_WAVEHIST;
      const uint32_t kind_lg = ((uint32_t)KIND_UNIFORM << 8) | (uint32_t)__builtin_ctz(P.rmax);
      st_agent(&P.slots[(uint64_t)k % P.nslot].tag, make_tag((uint64_t)k + 1, mode, kind_lg));
      __hip_atomic_fetch_add(&st->done, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  if (known & kWalkAfter) return;   // the walk_kernel launch after this one takes it in order
  order_global();     // every entry is in before the CAS below (so a failing CAS means the
  __syncthreads();    // sequencer's last look will find them)
  if (P.alarm_pct || P.criterion != HIST_CRIT_MAXBIN)
    sequence_stream<kSeqBatchExtra, true>(P, c, st);
  else
    sequence_stream<kSeqBatch, false>(P, c, st);
}

// Merge of a segment.
//
// flush_issue: sum the LDS table down to this thread's bin and add it, with no-return
// agent-scope atomics, into one of the segment's partial copies; thread 0 then takes a
// ticket (tiles done so far).  The caller reads the ticket when it next needs thread 0's
// results anyway; the workgroup that completed the segment's last tile runs
// finalize_segment.  A single-buffer launch takes no tickets: its last workgroup finalizes.
//
// finalize_segment does not rely on the other workgroups' atomics having landed before their
// tickets: it re-reads the copies until the 256 totals add up to the segment's byte count.
// Counts only grow and the exact total is known, so a matching sum means every
// contribution is in -- no per-flush acknowledgement wait is needed.
template <bool CLEAR = true>
__device__ __forceinline__ uint32_t flush_issue(uint32_t *lds, const Params &P, Ctl &c, uint32_t s, uint32_t kind,
                                                uint32_t lg, uint32_t nt, bool synced, bool ticket = true) {
  const uint32_t t = threadIdx.x;
  if (!synced) __syncthreads();   // the caller's barrier already ended every add otherwise
  TL(c, 9, s);
  const uint32_t h = table_bin<CLEAR>(lds, c, kind, lg);
  TL(c, 10, s);
  const uint32_t copies = 1u << P.clog2;
  uint32_t *part = P.partial + ((size_t)s << (P.clog2 + 8));
  // bins t and t + 1 (t even) go in one 64-bit atomic: half as many atomics, which the
  // memory side performs one queue at a time when the whole grid flushes together.  Each
  // 32-bit half only ever holds a count of this segment (< 2^32), so no carry crosses.
  const uint32_t hn = __shfl_xor(h, 1, 64);
  const uint64_t pair = (uint64_t)h | ((uint64_t)hn << 32);
  if (!(t & 1u) && pair)
    __hip_atomic_fetch_add(reinterpret_cast<uint64_t *>(&part[((blockIdx.x & (copies - 1u)) << 8) | t]), pair,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#ifdef HISTMI_STRICT_FENCES
  __threadfence();
#endif
  TL(c, 11, s);
  uint32_t before = 0;
  if (ticket && t == 0)
    before = __hip_atomic_fetch_add(&P.seg_done[s], nt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return before;
}

template <uint32_t NF = 8>
__device__ __forceinline__ void finalize_segment(const Params &P, Ctl &c, uint32_t s, const SegDesc &sd) {
  const uint32_t t = threadIdx.x;
  TL(c, 5, s);
  {
#ifdef HISTMI_STRICT_FENCES
    __threadfence();
#endif
    const uint32_t copies = 1u << P.clog2;
    uint32_t *part = P.partial + ((size_t)s << (P.clog2 + 8));
    uint32_t tot = 0;
    for (uint32_t tries = 0;; ++tries) {
      // read the copies NF at a time (all NF agent-scope loads in flight; the single-buffer
      // finalizer, which has no next tile's loads in registers, takes all 16 of its copies
      // in one memory round trip)
      tot = 0;
      if (copies >= NF) {
        for (uint32_t q = 0; q < copies; q += NF) {
          uint32_t x[NF];
#pragma unroll
          for (uint32_t u = 0; u < NF; ++u) x[u] = ld_agent(&part[((q + u) << 8) | t]);
#pragma unroll
          for (uint32_t u = 0; u < NF; ++u) tot += x[u];
        }
      } else if (copies >= 8) {
        for (uint32_t q = 0; q < copies; q += 8) {
          uint32_t x[8];
#pragma unroll
          for (uint32_t u = 0; u < 8; ++u) x[u] = ld_agent(&part[((q + u) << 8) | t]);
#pragma unroll
          for (uint32_t u = 0; u < 8; ++u) tot += x[u];
        }
      } else {
        for (uint32_t q = 0; q < copies; ++q) tot += ld_agent(&part[(q << 8) | t]);
      }
      if (block_sum_u64(tot, c) == sd.size) break;
      if (tries >= P.merge_polls) {   // never expected: contributions that do not land
        if (t == 0) {
          atomicAdd(&P.diag[2], 1u);
          if (sd.chunk >= 0 || sd.chunk == kServerChunk)
            __hip_atomic_fetch_add(&P.st[sd.stream_idx].merge_timeouts, (uint64_t)1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    TL(c, 6, s);
    for (uint32_t q = 0; q < copies; ++q) st_agent(&part[(q << 8) | t], 0u);
    if (sd.out) *gmem(&sd.out[t]) = tot;
    if (sd.acc) __hip_atomic_fetch_add(gmem(&sd.acc[t]), (uint64_t)tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (sd.chunk >= 0) stream_epilogue(P, c, sd.stream_idx, (int64_t)P.chunk_base + sd.chunk, tot, sd.size, sd.known);
    else if (sd.chunk == kServerChunk) server_epilogue(P, c, sd.stream_idx, tot);
    if (t == 0) st_agent(&P.seg_done[s], 0u);
  }
  TL(c, 7, s);
}

template <int KIND>
__device__ __forceinline__ Adder<KIND> make_adder(const uint32_t *lds, const Params &P, const Ctl &c) {
  Adder<KIND> ad;
  const uint32_t lane = lane_id();
  const uint32_t tb = lds_addr_of(lds);
  ad.lane = lane;
  if (KIND == KIND_WAVE || KIND == KIND_WAVE_AGG) {
    ad.a = tb + (wave_id() << 10);
    ad.s = 0;
  } else if (KIND == KIND_UNIFORM) {
    ad.a = tb + ((lane & ((1u << c.lg) - 1u)) << 2);
    ad.s = c.lg + 2u;
  } else {
    const uint32_t rr_lg = P.look_rr_lg;
    ad.a = tb + (P.look_off << 2) + ((lane & ((1u << rr_lg) - 1u)) << 2);
    ad.s = rr_lg + 2u;
  }
  return ad;
}

// Decision tag of segment s's chunk in an ordered stream launch, loaded by thread 0 without
// waiting, so that its round trip overlaps the other loads of a segment switch (0: nothing
// to load, or another thread).
__device__ __forceinline__ uint64_t tag_prefetch(const Params &P, uint32_t s) {
  if (!P.ordered || threadIdx.x != 0) return 0;
  const int64_t j = (int64_t)P.chunk_base + (int64_t)s - 1 - (int64_t)P.lag;
  if (j < 0) return 0;
  return ld_agent(&P.slots[(uint64_t)j % P.nslot].tag);
}

// One buffer spread over the whole grid (single launches): every workgroup strides over the
// buffer and flushes once.
template <int U>
__device__ __forceinline__ void single_path(uint32_t *lds, const Params &P, Ctl &c) {
  if (blockIdx.x >= P.ntiles) return;
  const uint32_t t = threadIdx.x;
  const SegDesc sd = P.seg0;
  const uint32_t kind = begin_segment(lds, P, c, sd, tag_prefetch(P, 0));
  TL(c, 2, 0);
  const uint32_t lg = c.lg;
  if (kind == KIND_WAVE) run_strided<KIND_WAVE, U>(lds, P, make_adder<KIND_WAVE>(lds, P, c), sd.ptr, sd.size);
  else if (kind == KIND_WAVE_AGG) run_strided<KIND_WAVE_AGG, U>(lds, P, make_adder<KIND_WAVE_AGG>(lds, P, c), sd.ptr, sd.size);
  else if (kind == KIND_UNIFORM) run_strided<KIND_UNIFORM, U>(lds, P, make_adder<KIND_UNIFORM>(lds, P, c), sd.ptr, sd.size);
  else run_strided<KIND_LOOKUP, U>(lds, P, make_adder<KIND_LOOKUP>(lds, P, c), sd.ptr, sd.size);
  TL(c, 3, 0);
  // No ticket elects the finalizer: the grid's last workgroup (the last dispatched, so
  // about the last to finish counting) finalizes once its own counts are flushed.  Its merge
  // re-reads the copies until they hold all n bytes, so it needs nothing from the others
  // but their atomics, and the others wait for nothing: the chain after the last count is
  // its atomics landing plus one re-read, not two returning atomics and then the read.
  flush_issue<false>(lds, P, c, 0, kind, lg, 0, false, false);   // its only flush: the table stays as it is
  TL(c, 4, 0);
  if (blockIdx.x + 1u == gridDim.x) {
    finalize_segment<16>(P, c, 0, sd);
    if (P.host_done) {
      // every thread's output and state writes reach memory that the host and the copy
      // engines read, then one store tells the host (the kernel has nothing left to do)
      __threadfence_system();
      __syncthreads();
      if (t == 0) __hip_atomic_store(P.host_done, P.done_seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// The segment descriptor is staged through LDS (c.sd[]) rather than held in registers: lanes
// 0..kSegWords-1 each load one word of it, so the load can be in flight across the flush of
// the previous segment without tying up scalar registers.
constexpr uint32_t kSegWords = sizeof(SegDesc) / 4;
__device__ __forceinline__ uint32_t seg_word(const Params &P, uint32_t s) {
  const uint32_t t = threadIdx.x;
  return t < kSegWords ? reinterpret_cast<const uint32_t *>(P.segs + s)[t] : 0u;
}
__device__ __forceinline__ void seg_stage(Ctl &c, uint32_t slot, uint32_t w) {
  if (threadIdx.x < kSegWords) reinterpret_cast<uint32_t *>(&c.sd[slot])[threadIdx.x] = w;
}

// Many segments cut into tiles (batches, stream pushes, server batches).  A workgroup takes
// its next tile when it starts a tile (dynamic: from an atomic counter, in launch order, so a
// workgroup waiting for an earlier chunk's decision only waits for tiles that running
// workgroups hold; static: the next tile of its contiguous range).  Halfway through the tile
// its control thread reads that tile's index and loads its record.  At the end of the tile
// the next tile's first loads are issued, and -- when the segment changes -- the next
// descriptor and decision tag are loaded while the workgroup flushes and takes its ticket,
// so a segment switch waits for about one memory round trip, with the data on its way.
template <int U>
__device__ __forceinline__ void multi_path(uint32_t *lds, const Params &P, Ctl &c) {
  const uint32_t t = threadIdx.x;
  uint32_t tile, tile_end = P.ntiles;
  uint32_t first_lo = 0, first_hi = 0, first_len = 0, first_seg = 0;   // static: the first tile
  // the first tile's round trip (a counter ticket, or the start record) is in flight while
  // the counting table is cleared
  if (P.dynamic) {
    uint32_t first = 0;
    if (t == 0) first = atomicAdd(&P.ctr[0], 1u);
    zero_table(lds, P);
    if (t == 0) c.next_tile = first;
    __syncthreads();
    tile = c.next_tile;
    __syncthreads();
  } else {
    // one memory round trip brings the workgroup's tile range, its first tile and that
    // tile's segment descriptor (one word per lane of the first wavefront)
    uint32_t w = 0;
    if (t < kStartWords) w = reinterpret_cast<const uint32_t *>(P.starts + blockIdx.x)[t];
    zero_table(lds, P);
    if (t < kStartWords) {
      if (t < 6) c.start[t] = w;
      else reinterpret_cast<uint32_t *>(&c.sd[0])[t - 6] = w;
    }
    __syncthreads();
    tile = __builtin_amdgcn_readfirstlane(c.start[0]);   // uniform: keep it in scalar registers
    tile_end = __builtin_amdgcn_readfirstlane(c.start[1]);
    first_lo = __builtin_amdgcn_readfirstlane(c.start[2]);
    first_hi = __builtin_amdgcn_readfirstlane(c.start[3]);
    first_len = __builtin_amdgcn_readfirstlane(c.start[4]);
    first_seg = __builtin_amdgcn_readfirstlane(c.start[5]);
  }
  const uint32_t rot = blockIdx.x * 7u;
  Pipe<U> a;
  Range rg;
  uint32_t cur = kNone, kind = KIND_WAVE, lg = 0, nt = 0;
  uint32_t sp = 0;    // c.sd[sp] describes the current segment
  uint32_t par = 0;   // parity of the tile step (c.ntile / c.nrec slot)
  if (tile < tile_end) {
    uint64_t hint;
    if (P.dynamic) {
      const TileRec r0 = P.recs[tile];
      const uint32_t w = seg_word(P, r0.seg);
      hint = tag_prefetch(P, r0.seg);
      rg = prime_range<U>(a, r0.addr, r0.len, rot);
      cur = r0.seg;
      seg_stage(c, sp, w);
      __syncthreads();
    } else {
      rg = prime_range<U>(a, (uint64_t)first_lo | ((uint64_t)first_hi << 32), first_len, rot);
      cur = first_seg;
      hint = 0;   // loaded where it is used: a prefetch here costs the kernel its fourth wave per SIMD
    }
    kind = begin_segment(lds, P, c, c.sd[sp], hint);
    TL(c, 2, cur);
    lg = c.lg;
  }
  while (tile < tile_end) {
    uint32_t req = tile + 1;
    if (P.dynamic && t == 0) req = atomicAdd(&P.ctr[0], 1u);
    TileRec rn;
    rn.addr = 0;
    rn.len = 0;
    rn.seg = kNone;
    auto mid = [&]() {
      if (t == 0 && req < tile_end) rn = P.recs[req];
    };
    if (kind == KIND_WAVE) run_primed<KIND_WAVE, U>(make_adder<KIND_WAVE>(lds, P, c), rg, rot, a, mid);
    else if (kind == KIND_WAVE_AGG) run_primed<KIND_WAVE_AGG, U>(make_adder<KIND_WAVE_AGG>(lds, P, c), rg, rot, a, mid);
    else if (kind == KIND_UNIFORM) run_primed<KIND_UNIFORM, U>(make_adder<KIND_UNIFORM>(lds, P, c), rg, rot, a, mid);
    else run_primed<KIND_LOOKUP, U>(make_adder<KIND_LOOKUP>(lds, P, c), rg, rot, a, mid);
    TL(c, 3, cur);
    ++nt;
    // one barrier ends the tile: every add is done and the next tile is published (slot by
    // parity, so a wave still reading the previous step's slot is never overwritten)
    if (t == 0) {
      c.ntile[par] = req;
      c.nrec[par] = rn;
    }
    __syncthreads();
    const uint32_t nxt = c.ntile[par];
    const TileRec r = c.nrec[par];
    par ^= 1u;
    const bool has_nxt = nxt < tile_end;
    if (has_nxt) rg = prime_range<U>(a, r.addr, r.len, rot);   // in flight during the switch
    const uint32_t ns = has_nxt ? r.seg : kNone;
    if (ns != cur) {
      uint32_t w = 0;
      uint64_t hint = 0;
      if (has_nxt) {
        w = seg_word(P, ns);
        hint = tag_prefetch(P, ns);
      }
      const uint32_t before = flush_issue(lds, P, c, cur, kind, lg, nt, true);
      // a second barrier publishes the ticket's verdict together with the next descriptor
      // (staged in the other slot, so a finalizer still reading c.sd[sp] is unaffected)
      if (t == 0) c.flag = (before + nt == c.sd[sp].ntiles) ? 1u : 0u;
      if (has_nxt) seg_stage(c, sp ^ 1u, w);
      __syncthreads();
      TL(c, 4, cur);
      if (c.flag) finalize_segment(P, c, cur, c.sd[sp]);
      if (has_nxt) {
        sp ^= 1u;
        cur = ns;
        nt = 0;
        kind = begin_segment(lds, P, c, c.sd[sp], hint);   // ends with the third barrier
        TL(c, 2, cur);
        lg = c.lg;
      }
    }
    tile = nxt;
  }
  if (P.dynamic) {
    __syncthreads();
    if (t == 0) {
      const uint32_t e = atomicAdd(&P.ctr[1], 1u);
      if (e == gridDim.x - 1) {
        st_agent(&P.ctr[0], 0u);
        st_agent(&P.ctr[1], 0u);
      }
    }
  }
}

// Load one word of each hot line of the kernel arguments at entry: the five scalar-cache
// misses then overlap, and every later read of an argument hits (otherwise each branch's
// first argument read waits for its own miss, one after another).  The words are read
// through the argument segment's base (Params is the kernel's only argument, at offset 0)
// and only fed to an empty asm, so no argument value is kept live from here.
__device__ __forceinline__ void touch_params() {
  static_assert(offsetof(Params, pat_words) <= 64 * kHotParamLines, "the hot fields fill the first lines");
  typedef const uint32_t __attribute__((address_space(4))) karg_word;
  const karg_word *k = (const karg_word *)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" ::"s"(k[0]), "s"(k[16]), "s"(k[32]), "s"(k[48]), "s"(k[64]));
}

template <int U>
__global__ void __launch_bounds__(kBlock) hist_main(const Params P) {
  // one dynamic LDS block: the counting table at address 0 (so table addresses need no
  // base offset), the lookup table after it, the control block at the end
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  touch_params();
  Ctl &c = *reinterpret_cast<Ctl *>(lds + P.table_words + P.look_words);
#ifdef HISTMI_TIMELINE
  if (threadIdx.x == 0) c.tl_n = 0;
#endif
  TL(c, 0, 0);
  if (P.single) single_path<U>(lds, P, c);
  else multi_path<U>(lds, P, c);
  TL(c, 8, 0);
}

// Rule P as a stand-alone call: one workgroup reads a uint64[256] histogram and writes a
// hist_pattern_t.
__global__ void __launch_bounds__(kBlock) pattern_update_kernel(const uint64_t *h, uint32_t S, uint32_t rmax,
                                                                 hist_pattern_t *out) {
  __shared__ Ctl c;
  const uint32_t t = threadIdx.x;
  const uint64_t v = h[t];
  const uint64_t N = block_sum_u64(v, c);
  uint32_t kind_lg;
  out->word[t] = rule_p_word(v, N, S, rmax, c, &kind_lg);
  if (t == 0) {
    out->total_S = S;
    out->rmax = rmax;
  }
}

// ------------------------------------------------------------------ read-bandwidth probe
//
// The HBM read roofline the counting kernels are measured against: every 16-byte vector of
// a buffer is loaded once (global_load_dwordx4, four per lane in flight, grid-stride) and its
// four 32-bit words are summed, so the loads cannot be dropped.  One u64 atomic per wavefront.
__global__ void __launch_bounds__(kBlock) read_probe_kernel(gu32x4 *v, uint64_t nvec, uint64_t *sum) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  uint64_t acc = 0;
  for (; i + 3 * stride < nvec; i += 4 * stride) {
    u32x4 x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = __builtin_nontemporal_load(v + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += (uint64_t)x[u][0] + x[u][1] + x[u][2] + x[u][3];
  }
  for (; i < nvec; i += stride) {
    const u32x4 x = __builtin_nontemporal_load(v + i);
    acc += (uint64_t)x[0] + x[1] + x[2] + x[3];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += shfl_xor_u64(acc, o);
  if (lane_id() == 0 && acc) atomicAdd(reinterpret_cast<unsigned long long *>(sum), (unsigned long long)acc);
}

// The in-order walk of a stream whose chunks left it to a later launch (kWalkAfter): one
// sequencer attempt, as a chunk's finalizer would make, once every chunk of the launch before
// it is in the ring.  A walk that finds the lock held leaves; the holder's last look then
// finds these chunks (see sequence_stream).  Change detection is on for such streams, so the
// walk takes the instantiation that can raise alarms, eight chunks per batch.
__global__ void __launch_bounds__(kBlock) walk_kernel(const Params P) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  Ctl &c = *reinterpret_cast<Ctl *>(lds);
#ifdef HISTMI_TIMELINE
  if (threadIdx.x == 0) c.tl_n = 0;
#endif
  // Walk this launch's chunks only, once the walk before it is done: its own push's chunks
  // are all in the ring, and the next push's walk takes the rest (a walk that took both
  // would hold up the counting launch queued behind it on its HIP stream).  The walk of the
  // push before comes first in whatever hardware queue this one shares with it, so the wait
  // ends; it is bounded all the same, and if it gives up (counted as a decision wait) this
  // walk falls back to walking whatever it finds, as a chunk's finalizer would.
  StreamDev *st = P.st;
  const uint64_t k0 = P.chunk_base;
  uint64_t stop = k0 + P.nseg;
  if (threadIdx.x == 0) {
    uint32_t i = 0;
    for (; i < P.wait_polls; ++i) {
      if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= k0 &&
          __hip_atomic_load(&st->seq_lock, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
        break;
      __builtin_amdgcn_s_sleep(8);
    }
    c.flag = i < P.wait_polls ? 1u : 0u;
    if (!c.flag) {
      atomicAdd(&P.diag[1], 1u);
      __hip_atomic_fetch_add(&st->wait_timeouts, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
  if (!c.flag) stop = ~0ull;
  __syncthreads();
  sequence_stream<kWalkBatch, true, true>(P, c, st, stop);
}

// A window stream's window after launches that did not walk it in order (their chunks left
// their histograms and sizes in the ring, see stream_epilogue): MW is the sum of the last W
// chunks' histograms and N their bytes (Sec. III.B), and the walk resumes at chunk n.  One
// workgroup, thread t holds bin t; it runs after those launches, so plain accesses suffice.
__global__ void __launch_bounds__(kBlock) window_rebuild_kernel(StreamDev *st, uint64_t n) {
  const uint32_t t = threadIdx.x;
  const uint32_t W = st->W, R = st->R;
  const uint64_t *ring = st->ring;
  const uint64_t *ring_n = st->ring_n;
  uint64_t mw = 0, N = 0;
  for (uint64_t q = n > W ? n - W : 0; q < n; ++q) {
    const uint32_t slot = (uint32_t)(q % R);
    mw += (uint32_t)ring[(size_t)slot * 256u + t];
    N += ring_n[slot] & kSizeMask;
  }
  st->mw[t] = mw;
  if (t == 0) {
    st->win_n = N;
    st->done = n;
  }
}

// ------------------------------------------------------------------ host-side launchers

uint32_t ctl_bytes() { return (uint32_t)((sizeof(Ctl) + 15) & ~(size_t)15); }

hipError_t launch_hist(const Params &P, const LaunchShape &sh, hipStream_t s, hipEvent_t done) {
  if (done) {
    // the event completes with the kernel's own dispatch: no marker packet between launches
    hipExtLaunchKernelGGL(hist_main<4>, dim3(sh.grid), dim3(kBlock), sh.lds_bytes, s, nullptr, done, 0u, P);
  } else {
    hipLaunchKernelGGL(hist_main<4>, dim3(sh.grid), dim3(kBlock), sh.lds_bytes, s, P);
  }
  return hipGetLastError();
}

hipError_t launch_pattern_update(const uint64_t *h, uint32_t S, uint32_t rmax, hist_pattern_t *out, hipStream_t s) {
  hipLaunchKernelGGL(pattern_update_kernel, dim3(1), dim3(kBlock), 0, s, h, S, rmax, out);
  return hipGetLastError();
}

hipError_t launch_walk(const Params &P, hipStream_t s) {
  hipLaunchKernelGGL(walk_kernel, dim3(1), dim3(kBlock), ctl_bytes(), s, P);
  return hipGetLastError();
}

hipError_t launch_window_rebuild(StreamDev *st, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(window_rebuild_kernel, dim3(1), dim3(kBlock), 0, s, st, n);
  return hipGetLastError();
}

hipError_t launch_read_probe(const void *d_in, uint64_t nvec, uint64_t *d_sum, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(read_probe_kernel, dim3(grid), dim3(kBlock), 0, s, (gu32x4 *)d_in, nvec, d_sum);
  return hipGetLastError();
}

hipError_t set_kernel_attrs(uint32_t max_dyn_lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&hist_main<4>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_dyn_lds);
}

hipError_t occupancy(uint32_t lds_bytes, int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void *>(&hist_main<4>),
                                                      kBlock, lds_bytes);
}

}  // namespace histmi

#ifdef HISTMI_TIMELINE
// Diagnostic build only (see include/histmi_timeline.h).
extern "C" hipError_t hist_timeline_shape(uint32_t *workgroups, uint32_t *per_workgroup) {
  if (!workgroups || !per_workgroup) return hipErrorInvalidValue;
  *workgroups = histmi::kTlWgs;
  *per_workgroup = histmi::kTlPer;
  return hipSuccess;
}
extern "C" hipError_t hist_timeline_read(uint64_t *host, size_t bytes) {
  if (!host || bytes != sizeof(histmi::g_timeline)) return hipErrorInvalidValue;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(histmi::g_timeline));
  if (e != hipSuccess) return e;
  return hipMemcpy(host, p, bytes, hipMemcpyDeviceToHost);
}
extern "C" hipError_t hist_timeline_reset(void) {
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(histmi::g_timeline));
  if (e != hipSuccess) return e;
  return hipMemset(p, 0, sizeof(histmi::g_timeline));
}
#endif
