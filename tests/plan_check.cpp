// Host-only checks of the tile planners (built and run by test_plan_cpu.py): every segment
// is covered exactly, in order, by its own contiguous tiles; inner tiles keep whole 16 KiB
// blocks and the size limit; static ranges are valid; and equal shares are balanced.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "runtime.h"

using namespace histmi;
using namespace histmi::rt;

static std::vector<SegDesc> segments(const std::vector<uint64_t> &sizes) {
  std::vector<SegDesc> segs(sizes.size());
  uint64_t addr = 1ull << 40;
  for (size_t j = 0; j < sizes.size(); ++j) {
    std::memset(&segs[j], 0, sizeof(SegDesc));
    segs[j].ptr = reinterpret_cast<const uint8_t *>(addr);
    segs[j].size = sizes[j];
    addr += sizes[j] + 4096;
  }
  return segs;
}

static bool covered(const std::vector<SegDesc> &segs, const MultiPlan &mp, uint64_t tile) {
  const TileRec *r = reinterpret_cast<const TileRec *>(mp.blob.data() + mp.seg_bytes);
  uint32_t next = 0;
  for (size_t j = 0; j < segs.size(); ++j) {
    if (segs[j].tile0 != next || segs[j].ntiles < 1) return false;
    uint64_t off = 0;
    for (uint32_t i = segs[j].tile0; i < segs[j].tile0 + segs[j].ntiles; ++i) {
      if (r[i].seg != j || r[i].addr != reinterpret_cast<uint64_t>(segs[j].ptr) + off || r[i].len > tile) return false;
      const bool last = i + 1 == segs[j].tile0 + segs[j].ntiles;
      if (!last && (r[i].len == 0 || r[i].len % 16384)) return false;
      off += r[i].len;
    }
    if (off != segs[j].size) return false;
    next = segs[j].tile0 + segs[j].ntiles;
  }
  return next == mp.ntiles;
}

// max over workgroups of (bytes + 64 KiB per segment touched) divided by the mean; 0 if invalid
static double split_case(const std::vector<uint64_t> &sizes, uint32_t maxg, uint64_t tile) {
  std::vector<SegDesc> segs = segments(sizes);
  MultiPlan mp;
  if (plan_split(segs, tile, maxg, &mp) != HIST_OK || !covered(segs, mp, tile)) return 0;
  uint64_t total = 0;
  for (uint64_t x : sizes) total += x;
  if (mp.blob.size() > plan_split_blob_max(sizes.size(), total, tile, maxg)) return 0;
  const TileRec *r = reinterpret_cast<const TileRec *>(mp.blob.data() + mp.seg_bytes);
  const uint32_t *b = reinterpret_cast<const uint32_t *>(mp.blob.data() + mp.seg_bytes + mp.rec_bytes);
  if (mp.grid < 1 || mp.grid > maxg || b[0] != 0 || b[mp.grid] != mp.ntiles) return 0;
  // each workgroup's start record: its range, its first tile and that tile's segment
  if (mp.start_off < mp.seg_bytes + mp.rec_bytes + (mp.grid + 1) * 4 || mp.start_off % 8 ||
      mp.blob.size() != mp.start_off + (size_t)mp.grid * sizeof(WgStart))
    return 0;
  const WgStart *st = reinterpret_cast<const WgStart *>(mp.blob.data() + mp.start_off);
  const SegDesc *sd = reinterpret_cast<const SegDesc *>(mp.blob.data());
  for (uint32_t w = 0; w < mp.grid; ++w) {
    if (st[w].tile != b[w] || st[w].tile_end != b[w + 1]) return 0;
    if (b[w] < b[w + 1] && (std::memcmp(&st[w].first, &r[b[w]], sizeof(TileRec)) != 0 ||
                            std::memcmp(&st[w].seg, &sd[r[b[w]].seg], sizeof(SegDesc)) != 0))
      return 0;
  }
  uint64_t mx = 0, sum = 0;
  for (uint32_t w = 0; w < mp.grid; ++w) {
    if (b[w] > b[w + 1]) return 0;
    uint64_t c = 0;
    uint32_t seg = ~0u;
    for (uint32_t i = b[w]; i < b[w + 1]; ++i) {
      c += r[i].len;
      if (r[i].seg != seg) c += 65536, seg = r[i].seg;
    }
    mx = std::max(mx, c);
    sum += c;
  }
  return sum ? (double)mx * mp.grid / (double)sum : 1.0;
}

static bool multi_case(const std::vector<uint64_t> &sizes, uint32_t maxg, uint64_t tile, uint32_t n_small = 0,
                       uint64_t small_tile = 0) {
  std::vector<SegDesc> segs = segments(sizes);
  MultiPlan mp;
  if (plan_multi(segs, tile, maxg, &mp, n_small, small_tile) != HIST_OK || !covered(segs, mp, tile) || mp.grid < 1 ||
      mp.grid > std::max<uint32_t>(1, maxg))
    return false;
  // the first n_small segments' tiles are at most small_tile (at least 16 KiB) long
  const TileRec *r = reinterpret_cast<const TileRec *>(mp.blob.data() + mp.seg_bytes);
  const uint64_t lim = std::max<uint64_t>(16384, std::min<uint64_t>(small_tile, std::max<uint64_t>(16384, tile)));
  for (uint32_t i = 0; i < mp.ntiles; ++i)
    if (small_tile && r[i].seg < n_small && r[i].len > lim) return false;
  return true;
}

// striped plans: workgroup w holds slice w of every segment, in segment order; each segment is
// covered exactly once, by slices of whole 16 KiB steps but its last; start records match
static bool striped_case(const std::vector<uint64_t> &sizes, uint32_t maxg) {
  std::vector<SegDesc> segs = segments(sizes);
  MultiPlan mp;
  if (plan_striped(segs, maxg, &mp) != HIST_OK || mp.grid < 1 || mp.grid > std::max<uint32_t>(1, maxg)) return false;
  const TileRec *r = reinterpret_cast<const TileRec *>(mp.blob.data() + mp.seg_bytes);
  const uint32_t *b = reinterpret_cast<const uint32_t *>(mp.blob.data() + mp.seg_bytes + mp.rec_bytes);
  const SegDesc *sd = reinterpret_cast<const SegDesc *>(mp.blob.data());
  const WgStart *st = reinterpret_cast<const WgStart *>(mp.blob.data() + mp.start_off);
  if (b[0] != 0 || b[mp.grid] != mp.ntiles) return false;
  std::vector<uint64_t> got(segs.size(), 0);
  std::vector<uint32_t> count(segs.size(), 0);
  std::vector<std::vector<std::pair<uint64_t, uint64_t>>> parts(segs.size());
  for (uint32_t w = 0; w < mp.grid; ++w) {
    if (b[w] > b[w + 1] || st[w].tile != b[w] || st[w].tile_end != b[w + 1]) return false;
    if (b[w] < b[w + 1] && (std::memcmp(&st[w].first, &r[b[w]], sizeof(TileRec)) != 0 ||
                            std::memcmp(&st[w].seg, &sd[r[b[w]].seg], sizeof(SegDesc)) != 0))
      return false;
    for (uint32_t i = b[w]; i < b[w + 1]; ++i) {
      if (i > b[w] && r[i].seg <= r[i - 1].seg) return false;   // segment order within a workgroup
      const uint32_t j = r[i].seg;
      const uint64_t off = r[i].addr - reinterpret_cast<uint64_t>(segs[j].ptr);
      if (off + r[i].len > segs[j].size) return false;
      if (off + r[i].len < segs[j].size && (r[i].len == 0 || r[i].len % 16384)) return false;
      parts[j].push_back({off, r[i].len});
      got[j] += r[i].len;
      ++count[j];
    }
  }
  for (size_t j = 0; j < segs.size(); ++j) {
    if (got[j] != segs[j].size || count[j] != segs[j].ntiles || sd[j].ntiles != segs[j].ntiles || count[j] < 1)
      return false;
    std::sort(parts[j].begin(), parts[j].end());
    uint64_t at = 0;
    for (auto &pr : parts[j]) {
      if (pr.first != at) return false;
      at += pr.second;
    }
  }
  return true;
}

// ---- forward progress of launches whose chunks wait for decisions (a model on the real plan)
//
// The kernel's rules, as the model takes them: a launch's tiles are handed out in order by
// one counter to whichever of its workgroups asks; a workgroup holds one tile at a time,
// waits (spinning, keeping its slot) until the decision its chunk runs with exists, counts,
// and asks again until the counter runs out, then leaves.  Chunk s of the stream runs with
// the decision made after chunk s - 1 - lag; that decision exists once every tile of that
// chunk is counted (W = 1; with a window, once every chunk up to it is -- `window` below).
// Two launches of the stream may be in flight and compete for the device's workgroup slots
// in any order; each launch's grid is the planner's.  `slots` is what the device holds.
struct Sim {
  std::vector<uint32_t> tile_seg;     // per launch-global tile: its chunk (stream index)
  std::vector<uint32_t> launch_of;    // per tile: 0 or 1
};

// Returns true if both launches finish; false if every resident workgroup waits on a
// decision that needs a tile no running workgroup can reach (a deadlock).  With
// `later_first` the dispatcher places every workgroup of the later launch before any of the
// earlier one's (as when the earlier launch's queue is still held by its own wait for the
// launch before it); otherwise it mixes them at random.
static bool simulate(const std::vector<uint64_t> &chunk_bytes, uint64_t tile, uint32_t grid_cap, uint32_t slots,
                     uint32_t lag, bool window, bool later_first, std::mt19937_64 &g, uint32_t n_small = 0,
                     uint64_t small_tile = 0, bool striped = false) {
  const uint32_t m = (uint32_t)chunk_bytes.size();
  struct L {
    MultiPlan mp;
    std::vector<SegDesc> segs;
    uint32_t next = 0, started = 0, left = 0;
  } ln[2];
  for (int l = 0; l < 2; ++l) {
    ln[l].segs = segments(chunk_bytes);
    if ((striped ? plan_striped(ln[l].segs, grid_cap, &ln[l].mp)
                 : plan_multi(ln[l].segs, tile, grid_cap, &ln[l].mp, n_small, small_tile)) != HIST_OK)
      return false;
    ln[l].left = ln[l].mp.grid;
  }
  const uint32_t nchunk = 2 * m;
  std::vector<uint32_t> tiles_left(nchunk);
  for (int l = 0; l < 2; ++l)
    for (uint32_t j = 0; j < m; ++j) tiles_left[l * m + j] = ln[l].segs[j].ntiles;
  auto chunk_done = [&](int64_t s) { return s < 0 || tiles_left[(size_t)s] == 0; };
  auto decided = [&](int64_t s) {   // the decision made after chunk s exists
    if (s < 0) return true;
    if (!window) return chunk_done(s);
    for (int64_t q = 0; q <= s; ++q)
      if (!chunk_done(q)) return false;
    return true;
  };
  struct WG {
    int l;
    uint32_t tile;   // held tile, or ~0u before the first request
    int work;        // remaining work units of the held tile once it runs
    uint32_t idx;    // striped: its index in its launch (its own range of tiles)
    uint32_t pos;    // striped: the next tile of that range
  };
  std::vector<const uint32_t *> bnd(2);
  for (int l = 0; l < 2; ++l)
    bnd[l] = reinterpret_cast<const uint32_t *>(ln[l].mp.blob.data() + ln[l].mp.seg_bytes + ln[l].mp.rec_bytes);
  std::vector<WG> res;   // resident workgroups
  uint32_t done_tiles = 0, total = ln[0].mp.ntiles + ln[1].mp.ntiles;
  std::vector<std::vector<uint32_t>> seg_of(2);
  for (int l = 0; l < 2; ++l) {
    const TileRec *r = reinterpret_cast<const TileRec *>(ln[l].mp.blob.data() + ln[l].mp.seg_bytes);
    for (uint32_t i = 0; i < ln[l].mp.ntiles; ++i) seg_of[l].push_back(r[i].seg);
  }
  for (long steps = 0; steps < 100000000L; ++steps) {
    if (done_tiles == total && res.empty() && ln[0].started == ln[0].mp.grid && ln[1].started == ln[1].mp.grid)
      return true;
    // the dispatcher places a pending workgroup of either launch in any order
    while (res.size() < slots && (ln[0].started < ln[0].mp.grid || ln[1].started < ln[1].mp.grid)) {
      int l = later_first ? 1 : (int)(g() & 1);
      if (ln[l].started == ln[l].mp.grid) l ^= 1;
      const uint32_t idx = ln[l].started++;
      res.push_back(WG{l, ~0u, 0, idx, striped ? bnd[l][idx] : 0u});
    }
    // some resident workgroup that can move makes its next move (tried in a random order)
    bool moved = false;
    std::vector<size_t> order(res.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::shuffle(order.begin(), order.end(), g);
    for (size_t i : order) {
      WG &w = res[i];
      L &x = ln[w.l];
      if (w.tile == ~0u) {   // ask for a tile (striped: take the next of its own range)
        const bool out = striped ? w.pos >= bnd[w.l][w.idx + 1] : x.next >= x.mp.ntiles;
        if (out) {
          res.erase(res.begin() + (long)i);   // out of tiles: leaves, freeing its slot
          moved = true;
          break;
        }
        w.tile = striped ? w.pos++ : x.next++;
        w.work = 1 + (int)(g() % 5);
        moved = true;
        break;
      }
      const int64_t s = (int64_t)w.l * m + seg_of[w.l][w.tile];
      if (!decided(s - 1 - (int64_t)lag)) continue;   // still waiting for its decision
      if (--w.work == 0) {
        --tiles_left[(size_t)s];
        ++done_tiles;
        w.tile = ~0u;
      }
      moved = true;
      break;
    }
    if (!moved) return false;   // every resident workgroup waits: deadlock
  }
  return false;
}

int main() {
  int bad = 0;
  // the single-stream workload: 66 chunks of 4 MiB over 512 workgroups
  const double head = split_case(std::vector<uint64_t>(66, 4u << 20), 512, 1u << 20);
  std::printf("headline balance %.4f\n", head);
  if (head == 0 || head > 1.03) bad = 1;
  // frames of one size, as many as workgroups: one frame each, no switch
  const double frames = split_case(std::vector<uint64_t>(512, 4u << 20), 512, 1u << 20);
  std::printf("frames balance %.4f\n", frames);
  if (frames != 1.0) bad = 1;
  if (split_case(std::vector<uint64_t>(3, 0), 512, 1u << 20) == 0) bad = 1;   // empty segments only
  if (split_case({1}, 1024, 16384) == 0 || split_case({100, 0, 7}, 1, 16384) == 0) bad = 1;
  std::mt19937_64 g(10110235);
  for (int it = 0; it < 3000 && !bad; ++it) {
    std::vector<uint64_t> s(1 + g() % 200);
    for (auto &x : s) {
      const int k = (int)(g() % 5);
      x = k == 0 ? 0 : k == 1 ? g() % 100 : k == 2 ? g() % (1u << 20) : g() % (16u << 20);
    }
    const uint32_t maxg = 1 + (uint32_t)(g() % 1200);
    const uint64_t tile = 16384ull * (1 + g() % 128);
    const uint32_t n_small = (uint32_t)(g() % (s.size() + 1));
    if (split_case(s, maxg, tile) == 0 || !multi_case(s, maxg, tile) ||
        !multi_case(s, maxg, tile, n_small, 16384ull * (1 + g() % 8)) || !striped_case(s, maxg)) {
      std::printf("invalid plan at case %d\n", it);
      bad = 1;
    }
  }
  // forward progress: with each launch's grid at most half of the device's slots (the rule
  // for launches that may wait), two launches of a stream always finish, whatever order the
  // dispatcher places their workgroups in and however fast each one counts; with grids that
  // fill the device, the later launch's waiting workgroups can hold every slot
  {
    std::mt19937_64 gs(20261203);
    int ok_half = 0, stalls_full = 0;
    const std::vector<uint64_t> chunks(24, 256u << 10);
    for (int it = 0; it < 300 && !bad; ++it) {
      const uint32_t slots = 16 + (uint32_t)(gs() % 48), lag = (uint32_t)(gs() % 4);
      const bool window = (gs() & 1) != 0, later_first = (gs() & 1) != 0;
      // tiles of 16-64 KiB; on half the runs the chunks that decide later chunks of the same
      // launch are cut into the smallest tiles (the planner's producer prefix)
      const uint64_t tile = 16384ull << (gs() % 3);
      const uint32_t m = (uint32_t)chunks.size();
      const uint32_t n_small = ((gs() & 1) != 0 && m > lag + 1) ? m - 1 - lag : 0u;
      if (simulate(chunks, tile, slots / 2, slots, lag, window, later_first, gs, n_small, 16384)) ++ok_half;
      else {
        std::printf("stall with half-capacity grids at case %d\n", it);
        bad = 1;
      }
      if (!simulate(chunks, tile, slots, slots, lag, window, later_first, gs, n_small, 16384)) ++stalls_full;
    }
    std::printf("progress model: %d of 300 runs finished at half capacity; %d of 300 stalled at full\n", ok_half,
                stalls_full);
    if (stalls_full == 0) bad = 1;   // the model must be able to show the hazard the rule avoids
    // striped static launches (every workgroup a slice of every chunk, in chunk order) at lag
    // 0 and 1: with each grid at most half of the slots, both launches always finish
    int ok_striped = 0;
    for (int it = 0; it < 300 && !bad; ++it) {
      const uint32_t slots = 16 + (uint32_t)(gs() % 48), lag = (uint32_t)(gs() % 2);
      const bool window = (gs() & 1) != 0, later_first = (gs() & 1) != 0;
      if (simulate(chunks, 16384, slots / 2, slots, lag, window, later_first, gs, 0, 0, true)) ++ok_striped;
      else {
        std::printf("stall of a striped launch with half-capacity grids at case %d\n", it);
        bad = 1;
      }
    }
    std::printf("striped progress model: %d of 300 runs finished at half capacity\n", ok_striped);
  }
  if (!striped_case(std::vector<uint64_t>(66, 4u << 20), 512) || !striped_case({0, 5, 0}, 3) ||
      !striped_case({1u << 20}, 1) || !striped_case(std::vector<uint64_t>(3, 0), 7)) {
    std::printf("invalid striped plan\n");
    bad = 1;
  }
  std::printf(bad ? "FAILED\n" : "all plans valid\n");
  return bad;
}
