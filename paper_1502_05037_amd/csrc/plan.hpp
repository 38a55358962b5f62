// Host half of the operator planner (the data split of eq. (2) and the gridding layout behind Φ and Φ†):
// fixed-point grid cells, the (tile, cell) order inside each block, work items, the per-stream row spans of the
// J = 8 gridder and the reduction chunks of the block norms of eq. (3).  Pure host code with no HIP runtime
// calls, so that it can also be built on its own (the sanitizer check of the tests does).
#pragma once

#include <hip/hip_runtime.h>   // uint2, int4

#include <cstdint>
#include <vector>

namespace sh {

constexpr int BALL_CHUNK = 8192;   // visibilities per reduction chunk

struct PlanShape {
  int64_t M;       // visibilities over all problems
  int K, log2K;    // oversampled grid side
  int T, log2T;    // tile side in cells
  int nT;          // tiles per grid side (K / T)
  int P, R;        // problems, blocks
  int chunk;       // most visibilities per work item
  int streams;     // streams per work item of the row-span gridder (0: no row spans; at most 8)
};

struct HostPlan {
  std::vector<uint2> coord;          // internal order: (cell << F | fraction) per axis, F = 32 - log2K
  std::vector<uint32_t> perm;        // internal position -> user index
  std::vector<int4> items;           // (global tile, first, count, patch slot)
  std::vector<int32_t> item_block;   // block of each item
  std::vector<int4> item_rows;       // per item: first row (bytes of x, y) and row count (bytes of z, w) per stream
  std::vector<int32_t> tile_items;   // slot range of each global tile (gtiles + 1)
  std::vector<int4> chunks;          // (block, first, end, 0) reduction chunks, never straddling a block
  std::vector<int32_t> chunk_first;  // first chunk of each block (R + 1)
  int max_items_per_tile = 0;
};

// Builds the plan of M visibilities `uv` (float64 (u, v) pairs in radians per pixel, user order) split into R
// blocks by `offs` (R + 1 ascending offsets, offs[0] = 0, offs[R] = M); block b belongs to problem
// block_prob[b].  The caller has validated the shape; nothing here allocates device memory.
void plan_host(const PlanShape& s, const double* uv, const int64_t* offs, const int32_t* block_prob, HostPlan& out);

}  // namespace sh
