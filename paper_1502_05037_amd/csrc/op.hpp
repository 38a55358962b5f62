// Internal layout of a measurement-operator plan (sh_op) and the launchers that use it.
#pragma once

#include "common.hpp"

// Kaiser-Bessel tap polynomials passed by value to the interpolation kernels: for tap t the weight
// at fraction f is sum_i c[t][i] s^i with s = 2f - 1 (degree KB_DEG).
#define KB_DEG 7
struct KBCoef {
  float c[16][KB_DEG + 1];
};

struct sh_op_s {
  int P = 1;                       // independent problems planned together (same n, alpha, J)
  std::vector<int64_t> vis_off;    // problem p owns visibilities [vis_off[p], vis_off[p+1])
  std::vector<int32_t> block_off;  // problem p owns blocks [block_off[p], block_off[p+1])
  std::vector<int32_t> block_prob; // problem of each block
  sh::DevBuf<int32_t> block_prob_d;
  int64_t M = 0;
  int n = 0, K = 0, log2K = 0, J = 0, alpha = 0, R = 0;
  int T = 0, log2T = 0, nT = 0;   // gridding tile side, tiles per grid side
  int chunk = 0;                   // most visibilities per work item
  double beta = 0;
  KBCoef kb{};
  std::vector<int64_t> offsets;    // block offsets (internal == user)
  sh::DevBuf<uint2> coord;         // internal order: fixed-point (grid cell << F | fraction), per axis
  sh::DevBuf<uint32_t> perm;       // internal index -> user index
  sh::DevBuf<int4> items;          // work items (tile, start, count, patch slot): sparse first, then dense
  // (start/count index internal order)
  sh::DevBuf<int32_t> tile_items;  // CSR over global tiles (problem * nT^2 + tile): patch slots of each tile
  int64_t n_items = 0, n_sparse = 0;
  int max_items_per_tile = 0;
  sh::DevBuf<float> deapod;        // 1 / psi_hat((r - n/2) / K), r < n
  sh::DevBuf<float2> tw;           // exp(-2 pi i m / K), m < K
  // scratch
  sh::DevBuf<float2> grid;         // P x K x K
  sh::DevBuf<float2> half;         // P x n x K
  sh::DevBuf<float2> patches;      // n_items x P x P
  sh::DevBuf<float2> vis_tmp;      // M
  // per-block reductions: chunks never straddle a block
  sh::DevBuf<int4> chunks;         // (block, start, end, 0)
  int64_t n_chunks = 0;
  std::vector<int32_t> chunk_first;  // host: first chunk of each block (R+1)
  sh::DevBuf<int32_t> chunk_first_d;
  sh::DevBuf<double> partials;     // 2 doubles per chunk
};

namespace sh {

// Phi / Phi^dagger on internal-order (or user-order, via the permutation) visibilities of all P
// problems; x holds P images.  Problem p's visibilities are scaled by scales[p] (device, NULL = 1).
sh_status phi_forward(sh_op op, const float* x, float2* vis, bool user_order, const float* scales, hipStream_t st);
sh_status phi_adjoint(sh_op op, const float2* vis, float* x, bool user_order, const float* scales, hipStream_t st);

// 2D FFT passes of the NUFFT over all P problems (fft.hip).
sh_status fft_forward_2d(sh_op op, const float* x, float2* grid, hipStream_t st);   // S, Z, F
sh_status fft_adjoint_2d(sh_op op, const float2* grid, float* x, hipStream_t st);   // F^H, Z^T, S, Re

}  // namespace sh
