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
  sh::DevBuf<int32_t> item_block;  // data block of each work item (order of `items`)
  // J = 8 gridder: per work item, the first cell row (tile-relative; bytes of x, y) and the number of cell
  // rows (bytes of z, w) of each of the streams the item is split into
  sh::DevBuf<int4> item_rows;
  sh::DevBuf<int32_t> tile_items;  // CSR over global tiles (problem * nT^2 + tile): patch slots of each tile
  int64_t n_items = 0, n_sparse = 0;
  int max_items_per_tile = 0;
  sh::DevBuf<float> deapod;        // 1 / psi_hat((r - n/2) / K), r < n
  sh::DevBuf<float> ones;          // n ones (FFT passes without deapodisation; set by the Toeplitz build)
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
// problems; x holds P images.  Block b's visibilities are scaled by scales[b] (device R floats, NULL = 1).
// With bmask (device R ints, NULL = all) only blocks b with bmask[b] != 0 take part: Phi leaves the other
// blocks' visibilities as they were, Phi^dagger reads only the selected blocks' visibilities.
sh_status phi_forward(sh_op op, const float* x, float2* vis, bool user_order, const float* scales, hipStream_t st,
                      const int32_t* bmask = nullptr);
sh_status phi_adjoint(sh_op op, const float2* vis, float* x, bool user_order, const float* scales, hipStream_t st,
                      const int32_t* bmask = nullptr);

// 2D FFT passes of the NUFFT over all P problems (fft.hip).
sh_status fft_forward_2d(sh_op op, const float* x, float2* grid, hipStream_t st);   // S, Z, F
sh_status fft_adjoint_2d(sh_op op, const float2* grid, float* x, hipStream_t st);   // F^H, Z^T, S, Re
// Unpruned forward 2D DFT of P dense K x K complex arrays, in place in buf (tmp: same size, clobbered).
sh_status fft_full_2d(sh_op op, float2* buf, float2* tmp, hipStream_t st);
// out = C * x per problem (linear 2D convolution of the n x n image x with the kernel whose DFT on
// the K x K grid is Ht, stored transposed: Ht[p][k2][k1]); tq: P x n x K complex scratch.
sh_status toeplitz_apply(sh_op op, const float* Ht, const float* x, float2* tq, float* out, hipStream_t st);

}  // namespace sh

// Toeplitz form of scale_p Re(Phi^H Phi) for a plan (toeplitz.hip).
struct sh_toep_s {
  sh::Arena arena;                 // a caller's workspace (sh_toeplitz_create_ws); declared first, freed last
  sh_op op = nullptr;
  sh::DevBuf<float> Ht;            // P x K x K: kernel spectrum / K^2 * scale_p, transposed
  sh::DevBuf<float2> tq;           // P x n x K scratch of the column pass
};

namespace sh {
// T = scale_p sum_b wblk_b^2 Re(Phi_b^H Phi_b) over the blocks b of problem p (scale, wblk: host arrays of P
// and R values, NULL = all 1).
sh_status toeplitz_build(sh_op op, const double* scale, const double* wblk, sh_toep_s* t, hipStream_t st);
// Multiplies problem p's operator by factor[p] (host P values).
sh_status toeplitz_rescale(sh_toep_s* t, const double* factor, hipStream_t st);
// Density estimate of 1 / ||Phi_b|| for every block b (blocknorm.hip).
sh_status block_density_weights(sh_op op, std::vector<double>& b, hipStream_t st);
}  // namespace sh
