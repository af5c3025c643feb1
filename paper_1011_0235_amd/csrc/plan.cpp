// Tile plans of multi-segment launches (host side): which tiles a launch has, and for
// static launches which workgroup runs which of them.
#include <algorithm>
#include <cstring>
#include <vector>

#include "runtime.h"

namespace histmi {
namespace rt {

// Tiles: each ends at its segment's end (n), at `tile` bytes (at most bytes / tile in all), or
// where a workgroup's share ends (each share end cuts at most once, since the cut moves past
// it): n + G + bytes / tile.  The grid is at most max_grid.
size_t plan_split_blob_max(uint64_t nseg, uint64_t bytes, uint64_t tile, uint32_t max_grid) {
  tile = std::max<uint64_t>(16384, std::min<uint64_t>(tile, 1ull << 30));
  const uint64_t G = std::max<uint32_t>(1, max_grid);
  const uint64_t recs = std::max<uint64_t>(nseg, 1) + G + bytes / tile + 1;
  return ((nseg * sizeof(SegDesc) + 15) & ~(uint64_t)15) + recs * sizeof(TileRec) + (((G + 1) * 4 + 15) & ~(uint64_t)15) +
         G * sizeof(WgStart);
}

hist_status_t plan_split(std::vector<SegDesc> &segs, uint64_t tile, uint32_t max_grid, MultiPlan *mp) {
  constexpr uint64_t kQuantum = 16384, kSwitchBytes = 65536;
  const uint32_t n = (uint32_t)segs.size();
  uint64_t total = 0, bytes = 0;
  for (uint32_t j = 0; j < n; ++j) {
    if (segs[j].size > kMaxSegBytes) return HIST_EOVERFLOW;
    if (segs[j].size && !segs[j].ptr) return HIST_EINVAL;
    total += segs[j].size + kSwitchBytes;
    bytes += segs[j].size;
  }
  tile = std::max<uint64_t>(kQuantum, std::min<uint64_t>(tile, 1ull << 30));
  const uint32_t G = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(max_grid, ceil_div(bytes, kQuantum)));
  auto share_end = [&](uint32_t g) { return g + 1 >= G ? total : total / G * (g + 1) + total % G * (g + 1) / G; };
  std::vector<TileRec> recs;
  std::vector<uint32_t> owner;
  recs.reserve((size_t)n + G + (size_t)(bytes / tile) + 1);
  owner.reserve(recs.capacity());
  uint64_t at = 0;   // the segment's start on the cost axis
  uint32_t g = 0;    // the workgroup whose share holds the current position
  for (uint32_t j = 0; j < n; ++j) {
    segs[j].tile0 = (uint32_t)recs.size();
    const uint64_t base = at + kSwitchBytes, sz = segs[j].size;
    uint64_t off = 0;
    do {   // an empty segment still gets one (empty) tile, so that it is finalized
      while (g + 1 < G && share_end(g) <= base + off) ++g;
      const uint64_t end = share_end(g);
      const uint64_t cut = end > base ? ceil_div(end - base, kQuantum) * kQuantum : off + kQuantum;
      const uint64_t len = std::min<uint64_t>({sz - off, tile, std::max<uint64_t>(cut, off + kQuantum) - off});
      recs.push_back(TileRec{reinterpret_cast<uint64_t>(segs[j].ptr) + off, (uint32_t)len, j});
      owner.push_back(g);
      off += len;
      if (recs.size() >= 0x7FFFFFFFull) return HIST_EOVERFLOW;
    } while (off < sz);
    segs[j].ntiles = (uint32_t)recs.size() - segs[j].tile0;
    at = base + sz;
  }
  const uint32_t ntiles = (uint32_t)recs.size();
  mp->nseg = n;
  mp->ntiles = ntiles;
  mp->grid = G;
  mp->seg_bytes = ((size_t)n * sizeof(SegDesc) + 15) & ~(size_t)15;
  mp->rec_bytes = (size_t)ntiles * sizeof(TileRec);
  const size_t bounds_bytes = (((size_t)G + 1) * 4 + 15) & ~(size_t)15;
  mp->start_off = mp->seg_bytes + mp->rec_bytes + bounds_bytes;
  mp->blob.assign(mp->start_off + (size_t)G * sizeof(WgStart), 0);
  std::memcpy(mp->blob.data(), segs.data(), (size_t)n * sizeof(SegDesc));
  std::memcpy(mp->blob.data() + mp->seg_bytes, recs.data(), mp->rec_bytes);
  uint32_t *bounds = reinterpret_cast<uint32_t *>(mp->blob.data() + mp->seg_bytes + mp->rec_bytes);
  // owners never decrease along the tiles: workgroup w runs tiles [bounds[w], bounds[w + 1])
  uint32_t i = 0;
  for (uint32_t w = 0; w <= G; ++w) {
    while (i < ntiles && owner[i] < w) ++i;
    bounds[w] = (w == G) ? ntiles : i;
  }
  WgStart *starts = reinterpret_cast<WgStart *>(mp->blob.data() + mp->start_off);
  for (uint32_t w = 0; w < G; ++w) {
    starts[w].tile = bounds[w];
    starts[w].tile_end = bounds[w + 1];
    if (bounds[w] < bounds[w + 1]) {
      starts[w].first = recs[bounds[w]];
      starts[w].seg = segs[recs[bounds[w]].seg];
    }
  }
  return HIST_OK;
}

hist_status_t plan_striped(std::vector<SegDesc> &segs, uint32_t max_grid, MultiPlan *mp) {
  constexpr uint64_t kQuantum = 16384;
  const uint32_t n = (uint32_t)segs.size();
  uint64_t most = 0;   // the most 16 KiB steps in one segment
  for (uint32_t j = 0; j < n; ++j) {
    if (segs[j].size > kMaxSegBytes) return HIST_EOVERFLOW;
    if (segs[j].size && !segs[j].ptr) return HIST_EINVAL;
    most = std::max<uint64_t>(most, ceil_div(segs[j].size, kQuantum));
  }
  const uint32_t G = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(max_grid, most));
  // segment j is cut into slices of q_j bytes (whole steps), slice w going to workgroup w;
  // an empty segment's one (empty) tile goes to workgroup 0
  std::vector<uint64_t> q(n);
  for (uint32_t j = 0; j < n; ++j) {
    q[j] = std::max<uint64_t>(kQuantum, ceil_div(ceil_div(segs[j].size, G), kQuantum) * kQuantum);
    if (q[j] > (1ull << 30)) return HIST_EOVERFLOW;   // a slice must fit a tile record
    segs[j].tile0 = 0;   // tiles of a segment are not contiguous here (unused by the kernel)
    segs[j].ntiles = segs[j].size ? (uint32_t)ceil_div(segs[j].size, q[j]) : 1u;
  }
  std::vector<TileRec> recs;
  std::vector<uint32_t> bounds(G + 1, 0);
  for (uint32_t w = 0; w < G; ++w) {
    bounds[w] = (uint32_t)recs.size();
    for (uint32_t j = 0; j < n; ++j) {
      const uint64_t off = (uint64_t)w * q[j], sz = segs[j].size;
      if (sz == 0 ? w == 0 : off < sz)
        recs.push_back(TileRec{reinterpret_cast<uint64_t>(segs[j].ptr) + off,
                               (uint32_t)(sz ? std::min<uint64_t>(q[j], sz - off) : 0u), j});
      if (recs.size() >= 0x7FFFFFFFull) return HIST_EOVERFLOW;
    }
  }
  bounds[G] = (uint32_t)recs.size();
  const uint32_t ntiles = (uint32_t)recs.size();
  mp->nseg = n;
  mp->ntiles = ntiles;
  mp->grid = G;
  mp->seg_bytes = ((size_t)n * sizeof(SegDesc) + 15) & ~(size_t)15;
  mp->rec_bytes = (size_t)ntiles * sizeof(TileRec);
  const size_t bounds_bytes = (((size_t)G + 1) * 4 + 15) & ~(size_t)15;
  mp->start_off = mp->seg_bytes + mp->rec_bytes + bounds_bytes;
  mp->blob.assign(mp->start_off + (size_t)G * sizeof(WgStart), 0);
  std::memcpy(mp->blob.data(), segs.data(), (size_t)n * sizeof(SegDesc));
  std::memcpy(mp->blob.data() + mp->seg_bytes, recs.data(), mp->rec_bytes);
  std::memcpy(mp->blob.data() + mp->seg_bytes + mp->rec_bytes, bounds.data(), ((size_t)G + 1) * 4);
  WgStart *starts = reinterpret_cast<WgStart *>(mp->blob.data() + mp->start_off);
  for (uint32_t w = 0; w < G; ++w) {
    starts[w].tile = bounds[w];
    starts[w].tile_end = bounds[w + 1];
    if (bounds[w] < bounds[w + 1]) {
      starts[w].first = recs[bounds[w]];
      starts[w].seg = segs[recs[bounds[w]].seg];
    }
  }
  return HIST_OK;
}

hist_status_t plan_multi(std::vector<SegDesc> &segs, uint64_t tile, uint32_t max_grid, MultiPlan *mp,
                         uint32_t n_small, uint64_t small_tile) {
  constexpr uint64_t kQuantum = 16384;
  const uint32_t n = (uint32_t)segs.size();
  tile = std::max<uint64_t>(kQuantum, std::min<uint64_t>(tile, 1ull << 30));
  small_tile = small_tile ? std::max<uint64_t>(kQuantum, std::min<uint64_t>(small_tile, tile)) : tile;
  uint64_t total = 0;
  for (uint32_t j = 0; j < n; ++j) {
    if (segs[j].size > kMaxSegBytes) return HIST_EOVERFLOW;
    if (segs[j].size && !segs[j].ptr) return HIST_EINVAL;
    total += segs[j].size;
  }
  std::vector<TileRec> recs;
  recs.reserve((size_t)n + (size_t)(total / tile) + 1);
  for (uint32_t j = 0; j < n; ++j) {
    segs[j].tile0 = (uint32_t)recs.size();
    const uint64_t sz = segs[j].size;
    uint64_t off = 0;
    const uint64_t tj = j < n_small ? small_tile : tile;
    do {   // an empty segment still gets one (empty) tile, so that it is finalized
      const uint64_t len = std::min<uint64_t>(tj, sz - off);
      recs.push_back(TileRec{reinterpret_cast<uint64_t>(segs[j].ptr) + off, (uint32_t)len, j});
      off += len;
      if (recs.size() >= 0x7FFFFFFFull) return HIST_EOVERFLOW;
    } while (off < sz);
    segs[j].ntiles = (uint32_t)recs.size() - segs[j].tile0;
  }
  const uint32_t ntiles = (uint32_t)recs.size();
  const uint32_t G = std::max<uint32_t>(1, std::min<uint32_t>(max_grid, ntiles));
  mp->nseg = n;
  mp->ntiles = ntiles;
  mp->grid = G;
  mp->seg_bytes = ((size_t)n * sizeof(SegDesc) + 15) & ~(size_t)15;
  mp->rec_bytes = (size_t)ntiles * sizeof(TileRec);
  // dynamic launches take tiles from the counter; the (unused) bounds are left zero
  mp->blob.assign(mp->seg_bytes + mp->rec_bytes + ((size_t)G + 1) * 4, 0);
  std::memcpy(mp->blob.data(), segs.data(), (size_t)n * sizeof(SegDesc));
  std::memcpy(mp->blob.data() + mp->seg_bytes, recs.data(), mp->rec_bytes);
  return HIST_OK;
}

}  // namespace rt
}  // namespace histmi
