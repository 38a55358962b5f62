// Per-block weights for normalising the data-fidelity splits of problem (3) block by block.
//
// Scaling the constraint of block i by any c_i > 0 (Phi_i -> c_i Phi_i, y_i -> c_i y_i, eps_i -> c_i eps_i)
// leaves its l2 ball, hence the solution set of (3), unchanged; SDMM's path depends on it through
// Q = 2I + sum_i c_i^2 Re(Phi_i^H Phi_i).  With one c for all blocks, a block whose ||Phi_i|| is small next
// to ||Phi|| (an outer uv annulus next to the dense centre) acts on x with a force scaled by
// (||Phi_i|| / ||Phi||)^2 and its constraint is met only after very many iterations.  Weights
// b_i ~ 1 / ||Phi_i|| give every block a comparable force.
//
// ||Phi_i||^2 is estimated from the density of the block's samples: for an n x n image, the largest
// eigenvalue of Re(Phi_i^H Phi_i) is close to n^2 times the largest number of the block's samples in a
// square window of side 2 pi / n in the uv plane (a uniform density rho per unit area gives the
// eigenvalue (2 pi)^2 rho).  The windows are those of alpha x alpha cells of the K x K grid (cell side
// 2 pi / K, K = alpha n), at every cell offset, periodic; cells are the planner's float64 cells.
//     lambda_i = n^2 max_window count_i,   b_i = 1 / sqrt(lambda_i).
#include <algorithm>
#include <cmath>

#include "op.hpp"

namespace {

// counts[b - g0][cell] += 1 for every visibility of the chunks of blocks g0.. (one work-group per chunk)
__global__ __launch_bounds__(256) void count_cells(const uint2* __restrict__ coord, const int4* __restrict__ chunks,
                                                   int c0, int g0, int log2K, uint32_t* __restrict__ counts) {
  const int4 c = chunks[c0 + blockIdx.x];
  const int F = 32 - log2K;
  uint32_t* h = counts + ((size_t)(c.x - g0) << (2 * log2K));
  for (int i = c.y + threadIdx.x; i < c.z; i += 256) {
    const uint2 q = coord[i];
    atomicAdd(&h[((size_t)(q.x >> F) << log2K) | (q.y >> F)], 1u);
  }
}

// mx[g0 + b] = max over cells (r, c) of the alpha x alpha window sum starting at (r, c), periodic; each
// work-group strides over the cells of block b = g0 + blockIdx.y, then one atomic max per work-group
__global__ __launch_bounds__(256) void window_max(const uint32_t* __restrict__ counts, int log2K, int alpha, int g0,
                                                  uint32_t* __restrict__ mx) {
  __shared__ uint32_t red[256];
  const int K = 1 << log2K, m = K - 1;
  const int64_t KK = int64_t(1) << (2 * log2K);
  const uint32_t* h = counts + ((size_t)blockIdx.y << (2 * log2K));
  uint32_t s = 0;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < KK; j += (int64_t)gridDim.x * 256) {
    const int r = int(j >> log2K), c = int(j & m);
    uint32_t w = 0;
    for (int a = 0; a < alpha; ++a)
      for (int d = 0; d < alpha; ++d) w += h[((size_t)((r + a) & m) << log2K) | ((c + d) & m)];
    s = max(s, w);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(&mx[g0 + blockIdx.y], red[0]);
}

}  // namespace

namespace sh {

sh_status block_density_weights(sh_op op, std::vector<double>& b, hipStream_t st) {
  const int R = op->R, K = op->K, n = op->n;
  const int64_t KK = int64_t(K) * K;
  // blocks per pass: at most 256 MiB of counters
  const int G = int(std::max<int64_t>(1, std::min<int64_t>(R, (int64_t(1) << 26) / KK)));
  sh::DevBuf<uint32_t> counts, mx;
  SH_TRY(counts.alloc(G * KK));
  SH_TRY(mx.alloc(R));
  SH_HIP(hipMemsetAsync(mx.ptr, 0, R * sizeof(uint32_t), st));
  for (int g0 = 0; g0 < R; g0 += G) {
    const int g1 = std::min(R, g0 + G);
    SH_HIP(hipMemsetAsync(counts.ptr, 0, size_t(g1 - g0) * KK * sizeof(uint32_t), st));
    const int c0 = op->chunk_first[g0], c1 = op->chunk_first[g1];
    if (c1 > c0) {
      hipLaunchKernelGGL(count_cells, dim3(unsigned(c1 - c0)), dim3(256), 0, st, op->coord.ptr, op->chunks.ptr, c0, g0,
                         op->log2K, counts.ptr);
      SH_LAUNCHED();
    }
    hipLaunchKernelGGL(window_max, dim3((unsigned)std::min<int64_t>(cdiv(KK, 256), 256), unsigned(g1 - g0)), dim3(256),
                       0, st, counts.ptr, op->log2K, op->alpha, g0, mx.ptr);
    SH_LAUNCHED();
  }
  std::vector<uint32_t> h(R);
  SH_HIP(hipMemcpyAsync(h.data(), mx.ptr, R * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  SH_HIP(hipStreamSynchronize(st));
  b.resize(R);
  for (int i = 0; i < R; ++i) {
    SH_REQUIRE(h[i] > 0, "block %d has no visibilities", i);
    b[i] = 1.0 / std::sqrt(double(n) * double(n) * double(h[i]));
  }
  return SH_OK;
}

}  // namespace sh

extern "C" {

sh_status sh_block_weights(sh_op op, double* b_out, void* stream) {
  SH_REQUIRE(op && b_out, "NULL argument");
  std::vector<double> b;
  SH_TRY(sh::block_density_weights(op, b, (hipStream_t)stream));
  std::copy(b.begin(), b.end(), b_out);
  return SH_OK;
}

}  // extern "C"
