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

static bool multi_case(const std::vector<uint64_t> &sizes, uint32_t maxg, uint64_t tile) {
  std::vector<SegDesc> segs = segments(sizes);
  MultiPlan mp;
  return plan_multi(segs, tile, maxg, &mp) == HIST_OK && covered(segs, mp, tile) && mp.grid >= 1 &&
         mp.grid <= std::max<uint32_t>(1, maxg);
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
    if (split_case(s, maxg, tile) == 0 || !multi_case(s, maxg, tile)) {
      std::printf("invalid plan at case %d\n", it);
      bad = 1;
    }
  }
  std::printf(bad ? "FAILED\n" : "all plans valid\n");
  return bad;
}
