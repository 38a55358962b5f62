// Host half of the operator planner: see plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace sh {

void plan_host(const PlanShape& s, const double* uv, const int64_t* offs, const int32_t* block_prob, HostPlan& out) {
  const int64_t M = s.M;
  const int K = s.K, F = 32 - s.log2K, log2T = s.log2T, nT = s.nT, T = s.T;
  const double scale = double(K) / (2.0 * M_PI);
  // fixed-point coordinates and the (tile, cell) key of every visibility, user order
  std::vector<uint2> cu(M);
  std::vector<uint32_t> key(M);
  for (int64_t m = 0; m < M; ++m) {
    uint32_t q[2];
    int cell[2];
    for (int ax = 0; ax < 2; ++ax) {
      const double kappa = uv[2 * m + ax] * scale;
      const double base = std::floor(kappa);
      const double frac = kappa - base;  // exact in float64, in [0, 1)
      int64_t cl = (int64_t)base % K;
      if (cl < 0) cl += K;
      uint64_t fr = (uint64_t)std::floor(std::ldexp(frac, F));
      if (F < 32 && fr >= (uint64_t(1) << F)) fr = (uint64_t(1) << F) - 1;
      q[ax] = (uint32_t)(((uint64_t)cl << F) | fr);
      cell[ax] = (int)cl;
    }
    cu[m] = make_uint2(q[0], q[1]);
    const uint32_t tile = uint32_t((cell[0] >> log2T) * nT + (cell[1] >> log2T));
    const uint32_t local = uint32_t(((cell[0] & (T - 1)) << log2T) | (cell[1] & (T - 1)));
    key[m] = (tile << (2 * log2T)) | local;
  }
  // internal order: sort by (tile, cell) inside each block (blocks never straddle problems); equal keys keep
  // their user order
  std::vector<uint32_t>& perm = out.perm;
  perm.assign(M, 0);
  std::vector<uint64_t> kv;
  for (int b = 0; b < s.R; ++b) {
    const int64_t lo = offs[b], hi = offs[b + 1];
    kv.resize(hi - lo);
    for (int64_t m = lo; m < hi; ++m) kv[m - lo] = (uint64_t(key[m]) << 32) | uint64_t(m - lo);
    std::sort(kv.begin(), kv.end());
    for (int64_t m = lo; m < hi; ++m) perm[m] = uint32_t(lo + (kv[m - lo] & 0xffffffffu));
  }
  out.coord.resize(M);
  for (int64_t i = 0; i < M; ++i) out.coord[i] = cu[perm[i]];
  // work items: runs of internal order with one (block, tile), cut into near-equal chunks of at most
  // `chunk`.  An item's tile id is global: problem * nT^2 + tile.  Patch slots follow (global tile,
  // block) order so that the fold finds the items of a tile in one contiguous slot range.
  const int ntiles = nT * nT;
  const int gtiles = s.P * ntiles;
  struct Item { int tile, start, count, block; };
  std::vector<Item> all;
  for (int64_t i = 0; i < M;) {
    const uint32_t k0 = key[perm[i]] >> (2 * log2T);
    const int b = int(std::upper_bound(offs, offs + s.R + 1, i) - offs) - 1;
    const int64_t bend = offs[b + 1];
    const int gt = block_prob[b] * ntiles + (int)k0;
    int64_t e = i;
    while (e < bend && (key[perm[e]] >> (2 * log2T)) == k0) ++e;
    const int64_t c = e - i, nck = (c + s.chunk - 1) / s.chunk;
    for (int64_t k = 0; k < nck; ++k) {
      const int64_t a = i + c * k / nck, bb = i + c * (k + 1) / nck;
      all.push_back({gt, (int)a, (int)(bb - a), b});
    }
    i = e;
  }
  std::vector<int> order(all.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return all[x].tile < all[y].tile; });
  std::vector<int32_t> per_tile(gtiles, 0), slot_of(all.size());
  out.tile_items.assign(gtiles + 1, 0);
  for (size_t q = 0; q < order.size(); ++q) {
    slot_of[order[q]] = (int32_t)q;
    per_tile[all[order[q]].tile]++;
  }
  for (int t = 0; t < gtiles; ++t) out.tile_items[t + 1] = out.tile_items[t] + per_tile[t];
  out.items.clear();
  out.item_block.clear();
  for (size_t q = 0; q < all.size(); ++q) {
    out.items.push_back(make_int4(all[q].tile, all[q].start, all[q].count, slot_of[q]));
    out.item_block.push_back(all[q].block);
  }
  // row-span gridder: the cell rows of each stream of each item.  The kernel splits an item into `streams`
  // runs of near-equal length, exactly as below; the first row and the row count of each are one byte each.
  out.item_rows.clear();
  if (s.streams > 0) {
    const int ns = s.streams;
    out.item_rows.resize(out.items.size());
    for (size_t q = 0; q < out.items.size(); ++q) {
      const int64_t a = out.items[q].y, c = out.items[q].z;
      uint32_t f[2] = {0u, 0u}, r[2] = {0u, 0u};
      for (int k = 0; k < ns; ++k) {
        const int64_t lo = a + c * k / ns, hi = a + c * (k + 1) / ns;
        uint32_t first = 0, rows = 1;      // an empty stream still owns one row
        if (hi > lo) {
          first = (key[perm[lo]] >> log2T) & uint32_t(T - 1);
          rows = ((key[perm[hi - 1]] >> log2T) & uint32_t(T - 1)) - first + 1;
        }
        f[k / 4] |= first << (8 * (k % 4));
        r[k / 4] |= rows << (8 * (k % 4));
      }
      out.item_rows[q] = make_int4((int)f[0], (int)f[1], (int)r[0], (int)r[1]);
    }
  }
  out.max_items_per_tile = gtiles > 0 ? *std::max_element(per_tile.begin(), per_tile.end()) : 0;
  // reduction chunks (never straddling a block)
  out.chunks.clear();
  out.chunk_first.assign(s.R + 1, 0);
  for (int b = 0; b < s.R; ++b) {
    out.chunk_first[b] = (int32_t)out.chunks.size();
    for (int64_t q = offs[b]; q < offs[b + 1]; q += BALL_CHUNK)
      out.chunks.push_back(make_int4(b, (int)q, (int)std::min<int64_t>(q + BALL_CHUNK, offs[b + 1]), 0));
  }
  out.chunk_first[s.R] = (int32_t)out.chunks.size();
}

}  // namespace sh
