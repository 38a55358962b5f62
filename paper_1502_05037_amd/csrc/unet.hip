// Learned warm start: a U-Net that maps the normalised dirty image to a first image estimate, with
// its training (forward, backward, Adam) on the GPU.
//
// Architecture (levels L, base channels c, c_l = c 2^(l-1)): encoder level l = two 3x3 convolutions
// (zero padding) + ReLU, levels 2..L preceded by a 2x2 max-pool; decoder level l = L-1..1: 2x2
// stride-2 transposed convolution c_{l+1} -> c_l, channel concat [upsampled, encoder output], two
// 3x3 convolutions + ReLU; head = 1x1 convolution to one channel + ReLU.  Loss: mean squared error
// between the head's output before its ReLU and the target (the ReLU applies to predictions).
//
// Number formats: fp32 master weights, gradients and Adam moments; bfloat16 weights, activations
// and incoming layer gradients as the operands of every matrix product; fp32 accumulation.
//
// Every convolution is a matrix product on the MFMA units (v_mfma_f32_16x16x32_bf16), activations NHWC
// (channels contiguous), a 3x3 convolution the product of im2col (K = 9 Cin, ordered (ky, kx, ci)) with the
// weight matrix.  Three forms:
//  * conv3_nt, the direct convolution, for inputs with a multiple of 32 channels (forward and input
//    gradients): per 32-channel chunk the input patch of an 8 x 32 pixel tile and the nine taps' weights are
//    staged in LDS once and each tap reads the patch at a constant offset; bf16 results leave through LDS in
//    16-byte stores, optionally also into a second buffer (the decoder's concatenation) and as the 2 x 2
//    max-pool of the tile.
//  * wgrad3, the direct weight gradient for the same layers: the gradient tile and the column-shifted input
//    patches are transposed into LDS so that the product contracts over pixels.
//  * gemm_nt / gemm_tn, products with im2col gathered inside the staging (the other layers, the transposed
//    convolutions, whose epilogue can write the upsampled pixels straight into the concatenation, and their
//    weight gradients): "NT" C[m][n] = sum_k A[m][k] B[n][k] with both operands contiguous along k (64 x 64
//    tiles, or 128 x 32 for at most 32 columns, k staged 64 at a time, optional split-K), "TN" contracting over
//    pixels with both operands transposed on the way into LDS and a column of ones for the bias gradient.
// The first layer (one input channel) and the 1 x 1 head are direct vector kernels.  Split-K partials are
// summed in a fixed order; results are deterministic.
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "op.hpp"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ uint16_t f2bf(float f) {   // nearest, ties to even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

inline unsigned nb(int64_t n, int t = 256) { return (unsigned)sh::cdiv(n, t); }
inline int64_t rup(int64_t v, int64_t m) { return sh::cdiv(v, m) * m; }

// 16-bit lanes of a 16-byte vector
__device__ __forceinline__ uint16_t u4_get(const uint4& v, int e) {
  const uint32_t w = e < 2 ? v.x : e < 4 ? v.y : e < 6 ? v.z : v.w;
  return (uint16_t)(w >> (16 * (e & 1)));
}
__device__ __forceinline__ uint4 u4_pack(const uint16_t* h) {
  return make_uint4(h[0] | (uint32_t(h[1]) << 16), h[2] | (uint32_t(h[3]) << 16), h[4] | (uint32_t(h[5]) << 16),
                    h[6] | (uint32_t(h[7]) << 16));
}

// ---------------------------------------------------------------------------------------------
// GEMM: C[m][n] = sum_{k in split z} A[m*lda + k] B[n*ldb + k] (+ bias[n]) (relu), bf16 operands.
// K is a multiple of 16.  Outputs: fp32 C (+ z*M*ldc for split partials) and/or bf16 Cb.
// ---------------------------------------------------------------------------------------------
constexpr int GBM = 64, GBN = 64, GBK = 64, GLD = GBK + 8;

// The next k-slab is loaded from global memory into registers while the MFMAs work on the current one
// from LDS (one LDS buffer, two barriers per slab).  Staging: thread t loads row t/4 of the A and B
// tiles, k-values 16 (t % 4) .. 16 (t % 4) + 15 (two 128-bit loads per operand).
// Implicit 3x3 im2col of an NHWC bf16 image as the A operand: row m = pixel (b, y, x) of a B x H x W
// batch, column k = (ky*3 + kx)*C + c < 9C takes the pixel (y+ky-1, x+kx-1), channel c (zero outside
// the image and for k >= 9C).  x has row stride ldx.
struct Im2col {
  const uint16_t* x;
  int ldx, H, W, C;
};
// Transposed-convolution output of a product (unused when dst is null): column n = (dy*2+dx)*Co + co of row m =
// input pixel (b, y, x) of a B x h x w batch goes, plus bias[co], as bf16 to channel co of the output pixel
// (2y+dy, 2x+dx) of the 2h x 2w image, rows of stride ld (Co and ld multiples of 8, dst 16-byte aligned)
struct Tconv {
  uint16_t* dst;
  int ld, h, w, Co;
};

template <bool GATHER, int WN>
__global__ __launch_bounds__(256) void gemm_nt(const uint16_t* __restrict__ A, int lda, const uint16_t* __restrict__ B,
                                               int ldb, int M, int N, int K, int kchunk,
                                               const float* __restrict__ bias, int relu, float* __restrict__ C,
                                               int ldc, uint16_t* __restrict__ Cb, int ldcb, Im2col g, Tconv tc,
                                               uint16_t* __restrict__ Cb2, int ldcb2) {
  // tile TM x TN (Cb2: optional second bf16 output, row stride ldcb2): 64 x 64 (four waves 2 x 2) or, for products with at most 32 columns, 128 x 32 (4 x 1)
  constexpr int TM = 128 / WN, TN = 32 * WN, AR = TM / 64, BU = TN / 32;
  __shared__ __attribute__((aligned(16))) uint16_t As[TM][GLD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][GLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // A: tile rows lr (+ 64), k-values lc .. lc + 15; B: rows br, k-values bc .. bc + 8 BU - 1
  const int lr = tid >> 2, lc = (tid & 3) * 16;
  const int br = BU == 2 ? lr : (tid >> 3), bc = BU == 2 ? lc : (tid & 7) * 8;
  uint4 ra[AR][2], rb[BU];
  // gather mode: the pixels of this thread's A rows
  int gb[AR], gy[AR], gx[AR];
#pragma unroll
  for (int r = 0; r < AR; ++r) {
    gb[r] = gy[r] = gx[r] = 0;
    if constexpr (GATHER) {
      const int m = m0 + lr + 64 * r;
      gb[r] = m / (g.H * g.W);
      const int rem = m - gb[r] * g.H * g.W;
      gy[r] = rem / g.W;
      gx[r] = rem - gy[r] * g.W;
    }
  }
  // Channel counts that are multiples of 8: the tap and channel of this thread's k-values lc + 8 e of the next
  // slab, advanced by GBK per slab (no integer division in the loop; C >= 8, so a slab moves at most GBK / C
  // taps)
  const bool fast = GATHER && (g.C & 7) == 0;
  int ktap[2] = {0, 0}, kch[2] = {0, 0};
  if (fast)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int k = kb + lc + 8 * e;
      ktap[e] = k / g.C;
      kch[e] = k - ktap[e] * g.C;
    }
  auto gather8 = [&](int r, int k, int e) -> uint4 {   // A[m0 + lr + 64 r][k .. k+7] of the implicit im2col
    if (fast) {
      const int tap = ktap[e];
      if (tap >= 9) return make_uint4(0, 0, 0, 0);
      const int ty = (tap * 11) >> 5, tx = tap - 3 * ty;   // tap / 3, tap % 3 for tap < 9
      const int sy = gy[r] + ty - 1, sx = gx[r] + tx - 1;
      if (sy < 0 || sy >= g.H || sx < 0 || sx >= g.W) return make_uint4(0, 0, 0, 0);
      return *(const uint4*)(g.x + ((int64_t)(gb[r] * g.H + sy) * g.W + sx) * g.ldx + kch[e]);
    }
    uint16_t v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int kq = k + q;
      v[q] = 0;
      if (kq < 9 * g.C) {
        const int tap = kq / g.C, c = kq - tap * g.C;
        const int sy = gy[r] + tap / 3 - 1, sx = gx[r] + tap % 3 - 1;
        if (sy >= 0 && sy < g.H && sx >= 0 && sx < g.W)
          v[q] = g.x[((int64_t)(gb[r] * g.H + sy) * g.W + sx) * g.ldx + c];
      }
    }
    return make_uint4(v[0] | (uint32_t(v[1]) << 16), v[2] | (uint32_t(v[3]) << 16), v[4] | (uint32_t(v[5]) << 16),
                      v[6] | (uint32_t(v[7]) << 16));
  };
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < AR; ++r)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int k = k0 + lc + 8 * e, m = m0 + lr + 64 * r;
        if constexpr (GATHER)
          ra[r][e] = (m < M && k < ke) ? gather8(r, k, e) : make_uint4(0, 0, 0, 0);
        else
          ra[r][e] = (m < M && k < ke) ? *(const uint4*)(A + (int64_t)m * lda + k) : make_uint4(0, 0, 0, 0);
      }
    if (fast)   // on to the next slab's k-values
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        kch[e] += GBK;
        while (kch[e] >= g.C) {
          kch[e] -= g.C;
          ++ktap[e];
        }
      }
#pragma unroll
    for (int e = 0; e < BU; ++e) {
      const int k = k0 + bc + 8 * e;
      rb[e] = (n0 + br < N && k < ke) ? *(const uint4*)(B + (int64_t)(n0 + br) * ldb + k) : make_uint4(0, 0, 0, 0);
    }
  };
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += GBK) {
#pragma unroll
    for (int r = 0; r < AR; ++r)
#pragma unroll
      for (int e = 0; e < 2; ++e) *(uint4*)&As[lr + 64 * r][lc + 8 * e] = ra[r][e];
#pragma unroll
    for (int e = 0; e < BU; ++e) *(uint4*)&Bs[br][bc + 8 * e] = rb[e];
    __syncthreads();
    if (k0 + GBK < ke) load(k0 + GBK);   // in flight during the products below
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 32) {
      const int ko = kk + 8 * (lane >> 4);
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8*)&As[wm * 32 + i * 16 + (lane & 15)][ko];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = *(const bf16x8*)&Bs[wn * 32 + j * 16 + (lane & 15)][ko];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D[i][j] of a 16x16 block: lane holds rows 4*(lane/16) + r, column lane%16
  if (tc.dst) {
    // transposed convolution: the bf16 tile goes through LDS (the A area, free after the last barrier) and
    // each input pixel's run of eight channels of one output pixel leaves in one 16-byte store
    constexpr int OP = TN + 8;
    static_assert(TM * OP <= TM * GLD, "output tile fits the A area");
    uint16_t* Ot = &As[0][0];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wn * 32 + j * 16 + (lane & 15), n = n0 + col;
      const float bv = n < N ? bias[n % tc.Co] : 0.f;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) Ot[(wm * 32 + i * 16 + 4 * (lane >> 4) + r) * OP + col] = f2bf(acc[i][j][r] + bv);
    }
    __syncthreads();
    constexpr int NG = TN / 8;
#pragma unroll
    for (int e = 0; e < TM * NG / 256; ++e) {
      const int gi = tid + 256 * e, row = gi / NG, c8 = gi - row * NG;
      const int m = m0 + row, n = n0 + 8 * c8;
      if (m >= M || n >= N) continue;
      const int q = n / tc.Co, co = n - q * tc.Co;
      const int b = m / (tc.h * tc.w), rem = m - b * tc.h * tc.w, y = rem / tc.w, x = rem - y * tc.w;
      const int64_t po = (int64_t)(b * 2 * tc.h + 2 * y + q / 2) * (2 * tc.w) + 2 * x + q % 2;
      *(uint4*)(tc.dst + po * tc.ld + co) = *(const uint4*)&Ot[row * OP + 8 * c8];
    }
    return;
  }
  if (C) C += (int64_t)blockIdx.z * M * ldc;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn * 32 + j * 16 + (lane & 15);
      if (n >= N) continue;
      const float bv = bias ? bias[n] : 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        if (m >= M) continue;
        float v = acc[i][j][r] + bv;
        if (relu) v = fmaxf(v, 0.f);
        if (C) C[(int64_t)m * ldc + n] = v;
        if (Cb) Cb[(int64_t)m * ldcb + n] = f2bf(v);
        if (Cb2) Cb2[(int64_t)m * ldcb2 + n] = f2bf(v);
      }
    }
}

// Direct 3x3 convolution of an NHWC bf16 image whose channel count C is a multiple of 32, as a product on the
// MFMA units: C[p][n] = sum_{c, tap} x[p + tap offset][c] Wop[n][tap*C + c] (+ bias[n]) (relu), the same
// product as gemm_nt over the implicit im2col (zero outside the image) with the k-sum taken channel chunk by
// channel chunk and tap by tap inside each chunk.  A work-group owns an 8 x 32 pixel tile of one image and TN
// (64 or 32) output channels; each of its four waves takes two tile rows (64 pixels) and all TN channels, as
// 4 x TN/16 blocks of v_mfma_f32_16x16x32_bf16.  Per chunk of 32 channels the 10 x 34 input patch and the nine
// taps' weight rows are staged in LDS once, and every tap's A operand is the patch read at a constant offset,
// so no gather arithmetic is repeated per tap and the weights are read once per 256 pixels.  The next chunk is
// loaded into registers while the current one is multiplied.  The MFMA operand and result layouts are those
// of gemm_nt.  Outputs: fp32 Cout (row stride ldc) and/or bf16 Cb (ldcb), optionally a second bf16 copy Cb2
// (ldcb2, e.g. the skip half of a concatenation); with `staged` (bf16 only, host-checked alignment) the tile
// leaves through LDS in 16-byte stores, and with Pout also as its 2 x 2 max-pool (Pidx: first-maximum index per
// window and channel, as pool_fwd).
template <int TN>
__global__ __launch_bounds__(256) void conv3_nt(const uint16_t* __restrict__ x, int ldx, int H, int W, int Cin,
                                                const uint16_t* __restrict__ Bw, int ldb, int N, int tiles_x,
                                                int tiles_img, const float* __restrict__ bias, int relu,
                                                float* __restrict__ Cout, int ldc, uint16_t* __restrict__ Cb,
                                                int ldcb, uint16_t* __restrict__ Cb2, int ldcb2, int staged,
                                                uint16_t* __restrict__ Pout, uint8_t* __restrict__ Pidx) {
  constexpr int TW = 32, TH = 8, BI = 4, BJ = TN / 16;
  constexpr int PW = TW + 2, NPIX = (TH + 2) * PW;
  constexpr int CS = 40;                           // LDS pitch of a pixel or weight row: 32 channels + 8
  constexpr int NPP = NPIX * 4, NWP = 9 * TN * 4;  // 16-byte pieces of the patch and of the weights
  constexpr int NA = (NPP + 255) / 256, NB = (NWP + 255) / 256;   // pieces per thread
  __shared__ __attribute__((aligned(16))) uint16_t Ps[NPIX * CS];
  __shared__ __attribute__((aligned(16))) uint16_t Ws[9 * TN * CS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bimg = blockIdx.x / tiles_img, t = blockIdx.x - bimg * tiles_img;
  const int ty0 = (t / tiles_x) * TH, tx0 = (t % tiles_x) * TW;
  const int n0 = blockIdx.y * TN;
  f32x4 acc[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // this thread's pieces: source offsets in elements without the chunk's channel offset (-1: zero, -2: none;
  // the host checks that the offsets fit in 30 bits)
  int sa[NA], sb[NB];
#pragma unroll
  for (int e = 0; e < NA; ++e) {
    const int pc = tid + 256 * e, pix = pc >> 2, part = pc & 3;
    const int py = pix / PW, px = pix - py * PW;
    const int y = ty0 - 1 + py, xx = tx0 - 1 + px;
    sa[e] = pc >= NPP ? -2 : (y >= 0 && y < H && xx >= 0 && xx < W) ? ((bimg * H + y) * W + xx) * ldx + 8 * part : -1;
  }
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    const int q = tid + 256 * e, part = q & 3, row = q >> 2;   // row = tap * TN + r
    const int tap = row / TN, r = row - tap * TN;
    sb[e] = q >= NWP ? -2 : n0 + r < N ? (n0 + r) * ldb + tap * Cin + 8 * part : -1;
  }
  uint4 ra[NA], rb[NB];
  auto load = [&](int c0) {
#pragma unroll
    for (int e = 0; e < NA; ++e) ra[e] = sa[e] >= 0 ? *(const uint4*)(x + sa[e] + c0) : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < NB; ++e) rb[e] = sb[e] >= 0 ? *(const uint4*)(Bw + sb[e] + c0) : make_uint4(0, 0, 0, 0);
  };
  // A rows of this lane (block i): tile pixel q = 64 wave + 16 i + lane % 16 (row 2 wave + i / 2), channels
  // 8 (lane / 16) ..; B rows: output channel 16 j + lane % 16
  const int abase = ((2 * wave) * PW + (lane & 15)) * CS + 8 * (lane >> 4);
  const int bbase = (lane & 15) * CS + 8 * (lane >> 4);
  load(0);
  for (int c0 = 0; c0 < Cin; c0 += 32) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int pc = tid + 256 * e;
      if (sa[e] != -2) *(uint4*)&Ps[(pc >> 2) * CS + 8 * (pc & 3)] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int q = tid + 256 * e;
      if (sb[e] != -2) *(uint4*)&Ws[(q >> 2) * CS + 8 * (q & 3)] = rb[e];
    }
    __syncthreads();
    if (c0 + 32 < Cin) load(c0 + 32);   // in flight during the products below
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int toff = ((tap / 3) * PW + tap % 3) * CS;
      bf16x8 a[BI], b[BJ];
#pragma unroll
      for (int i = 0; i < BI; ++i) a[i] = *(const bf16x8*)&Ps[abase + ((i >> 1) * PW + 16 * (i & 1)) * CS + toff];
#pragma unroll
      for (int j = 0; j < BJ; ++j) b[j] = *(const bf16x8*)&Ws[(tap * TN + 16 * j) * CS + bbase];
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D[i][j] of a 16x16 block: lane holds rows 4*(lane/16) + r, column lane%16
  if (staged) {
    // bf16 output only (the host checks N, ldcb, ldcb2 multiples of 8 and 16-byte aligned outputs): the tile goes
    // through LDS (the weight area, free after the last barrier) and leaves in 16-byte stores, each pixel's
    // channels contiguous; with Pout, also its 2 x 2 max-pool (first maximum's index in Pidx, as pool_fwd), every
    // window lying inside the tile (H and W even)
    constexpr int OP = TN + 8;   // pitch of a pixel's row (elements)
    static_assert(256 * OP <= 9 * TN * CS, "output tile fits the weight area");
#pragma unroll
    for (int j = 0; j < BJ; ++j) {
      const int n = n0 + j * 16 + (lane & 15);
      const float bv = (bias && n < N) ? bias[n] : 0.f;
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float v = acc[i][j][r] + bv;
          if (relu) v = fmaxf(v, 0.f);
          Ws[(64 * wave + 16 * i + 4 * (lane >> 4) + r) * OP + j * 16 + (lane & 15)] = f2bf(v);
        }
    }
    __syncthreads();
    constexpr int NG = TN / 8;   // groups of eight channels per pixel
#pragma unroll
    for (int e = 0; e < 256 * NG / 256; ++e) {
      const int g = tid + 256 * e, q = g / NG, c8 = g - q * NG;
      const int y = ty0 + q / TW, xx = tx0 + q % TW, n = n0 + 8 * c8;
      if (y >= H || xx >= W || n >= N) continue;
      const int64_t m = (int64_t)(bimg * H + y) * W + xx;
      const uint4 v = *(const uint4*)&Ws[q * OP + 8 * c8];
      *(uint4*)(Cb + m * ldcb + n) = v;
      if (Cb2) *(uint4*)(Cb2 + m * ldcb2 + n) = v;
    }
    if (Pout) {
      const int h2 = H / 2, w2 = W / 2;
#pragma unroll
      for (int e = 0; e < (TH / 2) * (TW / 2) * NG / 256; ++e) {
        const int g = tid + 256 * e, pq = g / NG, c8 = g - pq * NG;
        const int py = pq / (TW / 2), px = pq - py * (TW / 2);
        const int oy = ty0 / 2 + py, ox = tx0 / 2 + px, n = n0 + 8 * c8;
        if (oy >= h2 || ox >= w2 || n >= N) continue;
        uint4 v[4];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq)
          v[qq] = *(const uint4*)&Ws[((2 * py + qq / 2) * TW + 2 * px + qq % 2) * OP + 8 * c8];
        uint16_t bv[8];
        uint8_t bi[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          float best = -INFINITY;
          bi[c] = 0;
          bv[c] = 0;
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const uint16_t hv = u4_get(v[qq], c);
            const float f = bf2f(hv);
            if (f > best) {
              best = f;
              bi[c] = (uint8_t)qq;
              bv[c] = hv;
            }
          }
        }
        const int64_t o = ((int64_t)(bimg * h2 + oy) * w2 + ox) * N + n;
        *(uint4*)(Pout + o) = u4_pack(bv);
        *(uint2*)(Pidx + o) = make_uint2(bi[0] | (bi[1] << 8) | (bi[2] << 16) | (uint32_t(bi[3]) << 24),
                                         bi[4] | (bi[5] << 8) | (bi[6] << 16) | (uint32_t(bi[7]) << 24));
      }
    }
    return;
  }
  if (Cout && !Cb && !Cb2 && (N % 16) == 0 && (ldc % 4) == 0 && (reinterpret_cast<uintptr_t>(Cout) & 15) == 0) {
    // fp32 output only (the backward-data products): sixteen channels at a time through LDS (the weight area),
    // each pixel's sixteen values leaving in four 16-byte stores
    constexpr int OQ = 20;   // pitch of a pixel's row of sixteen floats
    static_assert(256 * OQ * 4 <= 9 * TN * CS * 2, "fp32 slice fits the weight area");
    float* Of = reinterpret_cast<float*>(Ws);
#pragma unroll
    for (int j = 0; j < BJ; ++j) {
      if (j > 0) __syncthreads();   // the previous slice has left
      const int n = n0 + j * 16 + (lane & 15);
      const float bv = (bias && n < N) ? bias[n] : 0.f;
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float v = acc[i][j][r] + bv;
          if (relu) v = fmaxf(v, 0.f);
          Of[(64 * wave + 16 * i + 4 * (lane >> 4) + r) * OQ + (lane & 15)] = v;
        }
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int g = tid + 256 * e, q = g >> 2, c4 = g & 3;
        const int y = ty0 + q / TW, xx = tx0 + q % TW, nn = n0 + j * 16 + 4 * c4;
        if (y >= H || xx >= W || nn >= N) continue;
        const int64_t m = (int64_t)(bimg * H + y) * W + xx;
        *(float4*)(Cout + m * ldc + nn) = *(const float4*)&Of[q * OQ + 4 * c4];
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < BJ; ++j) {
    const int n = n0 + j * 16 + (lane & 15);
    if (n >= N) continue;
    const float bv = bias ? bias[n] : 0.f;
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int y = ty0 + 2 * wave + (i >> 1), xx = tx0 + 16 * (i & 1) + 4 * (lane >> 4) + r;
        if (y >= H || xx >= W) continue;
        const int64_t m = (int64_t)(bimg * H + y) * W + xx;
        float v = acc[i][j][r] + bv;
        if (relu) v = fmaxf(v, 0.f);
        if (Cout) Cout[m * ldc + n] = v;
        if (Cb) Cb[m * ldcb + n] = f2bf(v);
        if (Cb2) Cb2[m * ldcb2 + n] = f2bf(v);
      }
  }
}

// out[i] = sum_z part[z*n + i], fixed order
__global__ void sum_splits(const float* __restrict__ part, int S, int64_t n, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  // eight partials loaded together, then added one after another: few outputs and many splits leave each
  // thread a long chain of loads, and the order of the sum stays z = 0, 1, ..., S-1
  float s = 0.f;
  int z = 0;
  for (; z + 8 <= S; z += 8) {
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = part[(z + e) * n + i];
#pragma unroll
    for (int e = 0; e < 8; ++e) s += v[e];
  }
  for (; z < S; ++z) s += part[z * n + i];
  out[i] = s;
}

// Columns k .. k+7 of the implicit 3x3 im2col row (see Im2col) of the pixel (b, y, x)
__device__ __forceinline__ uint4 im2col8(const Im2col& g, int b, int y, int x, int k) {
  if ((g.C & 7) == 0) {
    if (k >= 9 * g.C) return make_uint4(0, 0, 0, 0);
    const int tap = k / g.C, c = k - tap * g.C;
    const int sy = y + tap / 3 - 1, sx = x + tap % 3 - 1;
    if (sy < 0 || sy >= g.H || sx < 0 || sx >= g.W) return make_uint4(0, 0, 0, 0);
    return *(const uint4*)(g.x + ((int64_t)(b * g.H + sy) * g.W + sx) * g.ldx + c);
  }
  uint16_t v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int kq = k + q;
    v[q] = 0;
    if (kq < 9 * g.C) {
      const int tap = kq / g.C, c = kq - tap * g.C;
      const int sy = y + tap / 3 - 1, sx = x + tap % 3 - 1;
      if (sy >= 0 && sy < g.H && sx >= 0 && sx < g.W) v[q] = g.x[((int64_t)(b * g.H + sy) * g.W + sx) * g.ldx + c];
    }
  }
  return make_uint4(v[0] | (uint32_t(v[1]) << 16), v[2] | (uint32_t(v[3]) << 16), v[4] | (uint32_t(v[5]) << 16),
                    v[6] | (uint32_t(v[7]) << 16));
}

// Direct weight gradient of a 3x3 convolution whose input has a multiple of 32 channels C and whose output has a
// multiple of 32 channels M: part[z][m][tap*C + c] = sum_p g[p][m] x[p + tap offset][c] (x zero outside the
// image) and part[z][m][9C] = sum_p g[p][m] (the bias gradient), over the pixels of split z, in the layout of
// gemm_tn's partials (rows of N = 9C + 1).  A work-group owns 32 output channels (m0), 32 input channels (c0) and
// all nine taps over the 8 x 32 pixel tiles [t0, t1) of the batch; its four waves take (16-row block, 16-channel
// half) and the nine taps.  Per tile the gradient tile is transposed into LDS (pixels contiguous: the product
// contracts over pixels), and for each column shift kx the input patch, shifted by kx, likewise, so that every
// 16-byte operand read stays aligned; the three row shifts ky are then rows of the same patch.
__global__ __launch_bounds__(256) void wgrad3(const uint16_t* __restrict__ g, int ldg, const uint16_t* __restrict__ x,
                                              int ldx, int H, int W, int C, int M, int tiles_x, int tiles_img,
                                              int ntiles, int tiles_per_split, float* __restrict__ part) {
  constexpr int TW = 32, TH = 8, GP = 40;   // tile, pitch of a transposed row (32 pixels + 8)
  __shared__ __attribute__((aligned(16))) uint16_t Gt[32 * TH * GP];         // [m][ty][tx]
  __shared__ __attribute__((aligned(16))) uint16_t Xt[32 * (TH + 2) * GP];   // [c][py][tx]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rb = wave & 1, ch = wave >> 1;
  const int c0 = blockIdx.x * 32, m0 = blockIdx.y * 32, z = blockIdx.z;
  const int N = 9 * C + 1;
  const int tb = z * tiles_per_split, te = min(ntiles, tb + tiles_per_split);
  f32x4 acc[9], accb = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 ones;
#pragma unroll
  for (int e = 0; e < 8; ++e) ones[e] = (__bf16)1.0f;
  const bool bias = c0 == 0 && ch == 0;
  const int am = (rb * 16 + (lane & 15)) * TH * GP + 8 * (lane >> 4);   // + ty * GP
  const int bc = (ch * 16 + (lane & 15)) * (TH + 2) * GP + 8 * (lane >> 4);   // + py * GP
  for (int t = tb; t < te; ++t) {
    const int bimg = t / tiles_img, tl = t - bimg * tiles_img;
    const int ty0 = (tl / tiles_x) * TH, tx0 = (tl % tiles_x) * TW;
    bf16x8 a[TH];
#pragma unroll
    for (int kx = 0; kx < 3; ++kx) {
      __syncthreads();   // the previous round's operands have been read
      // pieces of two horizontally adjacent pixels and eight channels, written as one 32-bit word per channel;
      // consecutive lanes take consecutive pixel pairs, so a wave's words are contiguous in each row
      if (kx == 0) {
        // gradient tile: 128 pixel pairs x 4 groups of eight channels
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int q = tid + 256 * e, pr = q & 127, part8 = q >> 7;
          const int ty = pr / (TW / 2), tx = 2 * (pr % (TW / 2)), y = ty0 + ty, xx = tx0 + tx;
          uint4 v0 = make_uint4(0, 0, 0, 0), v1 = v0;
          const uint16_t* src = g + ((int64_t)(bimg * H + y) * W + xx) * ldg + m0 + 8 * part8;
          if (y < H && xx < W) v0 = *(const uint4*)src;
          if (y < H && xx + 1 < W) v1 = *(const uint4*)(src + ldg);
#pragma unroll
          for (int e2 = 0; e2 < 8; ++e2)
            *(uint32_t*)&Gt[((8 * part8 + e2) * TH + ty) * GP + tx] = u4_get(v0, e2) | (uint32_t(u4_get(v1, e2)) << 16);
        }
      }
      // input patch shifted by kx: rows ty0 - 1 .. ty0 + 8, columns tx0 - 1 + kx .. + 31 (160 pairs x 4 groups)
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const int q = tid + 256 * e;
        if (q >= 640) break;
        const int pr = q % 160, part8 = q / 160;
        const int py = pr / (TW / 2), tx = 2 * (pr % (TW / 2)), y = ty0 - 1 + py, xx = tx0 - 1 + kx + tx;
        uint4 v0 = make_uint4(0, 0, 0, 0), v1 = v0;
        const uint16_t* src = x + ((int64_t)(bimg * H + y) * W + xx) * ldx + c0 + 8 * part8;
        if (y >= 0 && y < H && xx >= 0 && xx < W) v0 = *(const uint4*)src;
        if (y >= 0 && y < H && xx + 1 >= 0 && xx + 1 < W) v1 = *(const uint4*)(src + ldx);
#pragma unroll
        for (int e2 = 0; e2 < 8; ++e2)
          *(uint32_t*)&Xt[((8 * part8 + e2) * (TH + 2) + py) * GP + tx] = u4_get(v0, e2) | (uint32_t(u4_get(v1, e2)) << 16);
      }
      __syncthreads();
      if (kx == 0) {
#pragma unroll
        for (int ty = 0; ty < TH; ++ty) a[ty] = *(const bf16x8*)&Gt[am + ty * GP];
        if (bias)
#pragma unroll
          for (int ty = 0; ty < TH; ++ty) accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ty], ones, accb, 0, 0, 0);
      }
      bf16x8 b[TH + 2];
#pragma unroll
      for (int py = 0; py < TH + 2; ++py) b[py] = *(const bf16x8*)&Xt[bc + py * GP];
#pragma unroll
      for (int ky = 0; ky < 3; ++ky)
#pragma unroll
        for (int ty = 0; ty < TH; ++ty)
          acc[ky * 3 + kx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ty], b[ty + ky], acc[ky * 3 + kx], 0, 0, 0);
    }
  }
  // D of a 16x16 block: lane holds rows 4*(lane/16) + r, column lane%16
  float* dst = part + (int64_t)z * M * N;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + rb * 16 + 4 * (lane >> 4) + r, c = c0 + ch * 16 + (lane & 15);
      dst[(int64_t)m * N + tap * C + c] = acc[tap][r];
    }
  if (bias && (lane & 15) == 0)
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[(int64_t)(m0 + rb * 16 + 4 * (lane >> 4) + r) * N + 9 * C] = accb[r];
}

// Weight-gradient products, which contract over pixels: C[m][n] = sum_{p in split z} A[p][m] Bv[p][n], p < P,
// with both operands read in their stored pixel-major layout and transposed on the way into LDS (the
// MFMA part is that of gemm_nt).  A: P x M, row stride lda.  Bv[p][n] = B[p][n] (row stride ldb) for
// n < NB, or the implicit 3x3 im2col of g.x when GATHER; 1 for n == NB when `ones` (the bias gradient);
// 0 beyond.  NB is a multiple of 8.  Staging: thread t takes pixels 2 (t % 32), 2 (t % 32) + 1 of the
// slab and the 8 columns 8 (t / 32) .. of each tile, and stores every column's pixel pair as one 32-bit
// LDS word (a wave's two column groups land in disjoint banks).
template <bool GATHER>
__global__ __launch_bounds__(256) void gemm_tn(const uint16_t* __restrict__ A, int lda, int M,
                                               const uint16_t* __restrict__ B, int ldb, int NB, int ones, int N, int P,
                                               int kchunk, float* __restrict__ C, int ldc, Im2col g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[GBM][GLD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GBN][GLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
  const int kb = blockIdx.z * kchunk, ke = min(P, kb + kchunk);
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int pp = 2 * (tid & 31), cc = 8 * (tid >> 5);
  const uint4 zero = make_uint4(0, 0, 0, 0);
  auto row8 = [&](const uint16_t* X, int ld, int p, int c0, int ncol) -> uint4 {   // X[p][c0 .. c0+7]
    if (c0 + 8 <= ncol && (ld & 7) == 0) return *(const uint4*)(X + (int64_t)p * ld + c0);
    uint16_t v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = c0 + q < ncol ? X[(int64_t)p * ld + c0 + q] : (uint16_t)0;
    return make_uint4(v[0] | (uint32_t(v[1]) << 16), v[2] | (uint32_t(v[3]) << 16), v[4] | (uint32_t(v[5]) << 16),
                      v[6] | (uint32_t(v[7]) << 16));
  };
  uint4 ra[2], rb[2];
  // gather mode: this thread's im2col columns n0 + cc .. + 7 are fixed (their tap and channel when C is a
  // multiple of 8), and its two pixels k0 + pp + e advance by GBK per slab: their (image, row, column) are
  // carried from slab to slab instead of divided out each time
  const bool fast = GATHER && (g.C & 7) == 0;
  const int ntap = fast ? (n0 + cc) / g.C : 0, nch = fast ? (n0 + cc) - ntap * g.C : 0;
  const int nty = (ntap * 11) >> 5, ntx = ntap - 3 * nty;   // ntap / 3, ntap % 3 for ntap < 9
  int pb[2] = {0, 0}, py[2] = {0, 0}, px[2] = {0, 0};
  if constexpr (GATHER)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int p = kb + pp + e;
      pb[e] = p / (g.H * g.W);
      const int rem = p - pb[e] * g.H * g.W;
      py[e] = rem / g.W;
      px[e] = rem - py[e] * g.W;
    }
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int p = k0 + pp + e;
      ra[e] = zero;
      rb[e] = zero;
      if (p >= ke) continue;
      if (m0 + cc < M) ra[e] = row8(A, lda, p, m0 + cc, M);
      const int n = n0 + cc;
      if (n < NB) {
        if constexpr (GATHER) {
          if (fast) {
            if (ntap < 9) {
              const int sy = py[e] + nty - 1, sx = px[e] + ntx - 1;
              if (sy >= 0 && sy < g.H && sx >= 0 && sx < g.W)
                rb[e] = *(const uint4*)(g.x + ((int64_t)(pb[e] * g.H + sy) * g.W + sx) * g.ldx + nch);
            }
          } else {
            rb[e] = im2col8(g, pb[e], py[e], px[e], n);
          }
        } else {
          rb[e] = row8(B, ldb, p, n, NB);
        }
      } else if (n == NB && ones) {
        rb[e] = make_uint4(0x3F80u, 0, 0, 0);   // bf16 1.0 in column NB
      }
    }
    if constexpr (GATHER)   // on to the next slab's pixels
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        px[e] += GBK;
        while (px[e] >= g.W) {
          px[e] -= g.W;
          if (++py[e] == g.H) {
            py[e] = 0;
            ++pb[e];
          }
        }
      }
  };
  auto half = [](const uint4& v, int j) -> uint32_t {   // 16-bit element j of v
    const uint32_t w = j < 2 ? v.x : j < 4 ? v.y : j < 6 ? v.z : v.w;
    return (j & 1) ? (w >> 16) : (w & 0xFFFFu);
  };
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += GBK) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      *(uint32_t*)&As[cc + j][pp] = half(ra[0], j) | (half(ra[1], j) << 16);
      *(uint32_t*)&Bs[cc + j][pp] = half(rb[0], j) | (half(rb[1], j) << 16);
    }
    __syncthreads();
    if (k0 + GBK < ke) load(k0 + GBK);   // in flight during the products below
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 32) {
      const int ko = kk + 8 * (lane >> 4);
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8*)&As[wm * 32 + i * 16 + (lane & 15)][ko];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = *(const bf16x8*)&Bs[wn * 32 + j * 16 + (lane & 15)][ko];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  C += (int64_t)blockIdx.z * M * ldc;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn * 32 + j * 16 + (lane & 15);
      if (n >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        if (m < M) C[(int64_t)m * ldc + n] = acc[i][j][r];
      }
    }
}

// ---- layout kernels ----------------------------------------------------------------------------

__global__ void f32_to_bf16(const float* __restrict__ in, uint16_t* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = f2bf(in[i]);
}

// 2x2 max-pool, NHWC; idx = row-major index of the first maximum of the window
__global__ void pool_fwd(const uint16_t* __restrict__ x, int B, int H, int W, int C, uint16_t* __restrict__ y,
                         uint8_t* __restrict__ idx) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int h = H / 2, w = W / 2;
  if (t >= (int64_t)B * h * w * C) return;
  const int c = int(t % C);
  const int64_t po = t / C;
  const int b = int(po / ((int64_t)h * w));
  const int rem = int(po - (int64_t)b * h * w);
  const int oy = rem / w, ox = rem - oy * w;
  float best = -INFINITY;
  int bi = 0;
  uint16_t bv = 0;
  for (int q = 0; q < 4; ++q) {
    const uint16_t v = x[((int64_t)(b * H + 2 * oy + q / 2) * W + 2 * ox + q % 2) * C + c];
    const float f = bf2f(v);
    if (f > best) {
      best = f;
      bi = q;
      bv = v;
    }
  }
  y[t] = bv;
  idx[t] = (uint8_t)bi;
}

// gradient of the pool: g_in (B, H, W, C) fp32 from g_out (B, H/2, W/2, C) fp32
__global__ void pool_bwd(const float* __restrict__ gout, const uint8_t* __restrict__ idx, int B, int H, int W, int C,
                         float* __restrict__ gin) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int h = H / 2, w = W / 2;
  if (t >= (int64_t)B * h * w * C) return;
  const int c = int(t % C);
  const int64_t po = t / C;
  const int b = int(po / ((int64_t)h * w));
  const int rem = int(po - (int64_t)b * h * w);
  const int oy = rem / w, ox = rem - oy * w;
  const int bi = idx[t];
  const float g = gout[t];
  for (int q = 0; q < 4; ++q)
    gin[((int64_t)(b * H + 2 * oy + q / 2) * W + 2 * ox + q % 2) * C + c] = q == bi ? g : 0.f;
}

// transposed-conv output: Y[p_in][(dy*2+dx)*Co + co] (fp32) + bias -> dst (2h x 2w, row stride ld), bf16
__global__ void tconv_scatter(const float* __restrict__ Y, const float* __restrict__ bias, int B, int h, int w, int Co,
                              uint16_t* __restrict__ dst, int ld) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)B * h * w * 4 * Co) return;
  const int n = int(t % (4 * Co));
  const int64_t p = t / (4 * Co);
  const int q = n / Co, co = n - q * Co;
  const int b = int(p / ((int64_t)h * w));
  const int rem = int(p - (int64_t)b * h * w);
  const int y = rem / w, x = rem - y * w;
  const int64_t po = (int64_t)(b * 2 * h + 2 * y + q / 2) * (2 * w) + 2 * x + q % 2;
  dst[po * ld + co] = f2bf(Y[t] + bias[co]);
}

// transposed-conv backward: gG[p_in][(dy*2+dx)*Co + co] = bf16(g[(2y+dy, 2x+dx)][co]) (g fp32, row stride ld)
__global__ void tconv_gather(const float* __restrict__ g, int ld, int B, int h, int w, int Co, uint16_t* __restrict__ gG) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)B * h * w * 4 * Co) return;
  const int n = int(t % (4 * Co));
  const int64_t p = t / (4 * Co);
  const int q = n / Co, co = n - q * Co;
  const int b = int(p / ((int64_t)h * w));
  const int rem = int(p - (int64_t)b * h * w);
  const int y = rem / w, x = rem - y * w;
  const int64_t po = (int64_t)(b * 2 * h + 2 * y + q / 2) * (2 * w) + 2 * x + q % 2;
  gG[t] = f2bf(g[po * ld + co]);
}


// gm[p][c] = bf16((g[p*ldg + c] (+ g2[p*ldg2 + c])) * (act[p][c] > 0))
__global__ void relu_mask_grad(const float* __restrict__ g, int ldg, const float* __restrict__ g2, int ldg2,
                               const uint16_t* __restrict__ act, int64_t P, int C, uint16_t* __restrict__ gm) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= P * C) return;
  const int64_t p = t / C;
  const int c = int(t - p * C);
  float v = g[p * ldg + c];
  if (g2) v += g2[p * ldg2 + c];
  gm[t] = bf2f(act[t]) > 0.f ? f2bf(v) : (uint16_t)0;
}

// ---- the layout kernels above, eight channels per thread (channel counts, row strides and channel offsets
// multiples of 8, 16-byte aligned buffers, fewer than 2^31 groups of eight); each element is computed as above
__device__ __forceinline__ void load8f(const float* p, float* v) {
  const float4 a = *(const float4*)p, b = *(const float4*)(p + 4);
  v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w, v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
}
__device__ __forceinline__ void store8f(float* p, const float* v) {
  *(float4*)p = make_float4(v[0], v[1], v[2], v[3]);
  *(float4*)(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
}

__global__ void pool_fwd8(const uint16_t* __restrict__ x, int B, int H, int W, int C, uint16_t* __restrict__ y,
                          uint8_t* __restrict__ idx) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int C8 = C >> 3, h = H / 2, w = W / 2;
  if (t >= B * h * w * C8) return;
  const int c8 = t % C8, po = t / C8;
  const int b = po / (h * w), rem = po - b * h * w, oy = rem / w, ox = rem - oy * w;
  uint4 v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = *(const uint4*)(x + ((int64_t)(b * H + 2 * oy + q / 2) * W + 2 * ox + q % 2) * C + 8 * c8);
  uint16_t bv[8];
  uint8_t bi[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float best = -INFINITY;
    bi[e] = 0;
    bv[e] = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint16_t hv = u4_get(v[q], e);
      const float f = bf2f(hv);
      if (f > best) {
        best = f;
        bi[e] = (uint8_t)q;
        bv[e] = hv;
      }
    }
  }
  const int64_t o = (int64_t)po * C + 8 * c8;
  *(uint4*)(y + o) = u4_pack(bv);
  *(uint2*)(idx + o) = make_uint2(bi[0] | (bi[1] << 8) | (bi[2] << 16) | (uint32_t(bi[3]) << 24),
                                  bi[4] | (bi[5] << 8) | (bi[6] << 16) | (uint32_t(bi[7]) << 24));
}

__global__ void pool_bwd8(const float* __restrict__ gout, const uint8_t* __restrict__ idx, int B, int H, int W, int C,
                          float* __restrict__ gin) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int C8 = C >> 3, h = H / 2, w = W / 2;
  if (t >= B * h * w * C8) return;
  const int c8 = t % C8, po = t / C8;
  const int b = po / (h * w), rem = po - b * h * w, oy = rem / w, ox = rem - oy * w;
  const int64_t o = (int64_t)po * C + 8 * c8;
  float g[8];
  load8f(gout + o, g);
  const uint2 ib = *(const uint2*)(idx + o);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float r[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = int(((e < 4 ? ib.x : ib.y) >> (8 * (e & 3))) & 255) == q ? g[e] : 0.f;
    store8f(gin + ((int64_t)(b * H + 2 * oy + q / 2) * W + 2 * ox + q % 2) * C + 8 * c8, r);
  }
}


__global__ void tconv_gather8(const float* __restrict__ g, int ld, int B, int h, int w, int Co,
                              uint16_t* __restrict__ gG) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int N8 = Co / 2;
  if (t >= B * h * w * N8) return;
  const int n = 8 * (t % N8), p = t / N8;
  const int q = n / Co, co = n - q * Co;
  const int b = p / (h * w), rem = p - b * h * w, y = rem / w, x = rem - y * w;
  const int64_t po = (int64_t)(b * 2 * h + 2 * y + q / 2) * (2 * w) + 2 * x + q % 2;
  float v[8];
  load8f(g + po * ld + co, v);
  uint16_t r[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = f2bf(v[e]);
  *(uint4*)(gG + 8 * (int64_t)t) = u4_pack(r);
}


__global__ void relu_mask_grad8(const float* __restrict__ g, int ldg, const float* __restrict__ g2, int ldg2,
                                const uint16_t* __restrict__ act, int P, int C, uint16_t* __restrict__ gm) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int C8 = C >> 3;
  if (t >= P * C8) return;
  const int p = t / C8, c = 8 * (t - p * C8);
  float v[8];
  load8f(g + (int64_t)p * ldg + c, v);
  if (g2) {
    float v2[8];
    load8f(g2 + (int64_t)p * ldg2 + c, v2);
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] += v2[e];
  }
  const uint4 a = *(const uint4*)(act + 8 * (int64_t)t);
  uint16_t r[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = bf2f(u4_get(a, e)) > 0.f ? f2bf(v[e]) : (uint16_t)0;
  *(uint4*)(gm + 8 * (int64_t)t) = u4_pack(r);
}

// 3x3 convolution of a one-channel bf16 image (the network's first layer): out[p][n] = relu(sum_tap x[p + tap
// offset] wf[n][tap] + bias[n]) with the taps in order and fp32 sums of the exact bf16 products.  One pixel
// and all N (a multiple of 8, at most 64) output channels per thread; the weights and biases are staged in LDS
// once per work-group and read there by every lane at the same address.  bf16 output of row stride ldo.
__global__ __launch_bounds__(256) void conv3_c1(const uint16_t* __restrict__ x, int ldx, int B, int H, int W,
                                                const uint16_t* __restrict__ wf, int Kp, int N,
                                                const float* __restrict__ bias, uint16_t* __restrict__ out, int ldo) {
  // rows of 12 (16-byte aligned: a channel's nine weights in three 16-byte reads, the last three zero)
  __shared__ __attribute__((aligned(16))) float ws[64 * 12];
  __shared__ float bs[64];
  for (int e = threadIdx.x; e < N * 12; e += 256) ws[e] = e % 12 < 9 ? bf2f(wf[(e / 12) * Kp + e % 12]) : 0.f;
  for (int e = threadIdx.x; e < N; e += 256) bs[e] = bias[e];
  __syncthreads();
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= B * H * W) return;
  const int b = p / (H * W), rem = p - b * H * W, y = rem / W, xx = rem - y * W;
  float xv[9];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int sy = y + tap / 3 - 1, sx = xx + tap % 3 - 1;
    xv[tap] = (sy >= 0 && sy < H && sx >= 0 && sx < W) ? bf2f(x[((int64_t)(b * H + sy) * W + sx) * ldx]) : 0.f;
  }
  for (int n0 = 0; n0 < N; n0 += 8) {
    uint16_t r[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float* wr = ws + (n0 + e) * 12;
      float acc = 0.f;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) acc = fmaf(xv[tap], wr[tap], acc);
      r[e] = f2bf(fmaxf(acc + bs[n0 + e], 0.f));
    }
    *(uint4*)(out + (int64_t)p * ldo + n0) = u4_pack(r);
  }
}

// The head's 1 x 1 convolution to one channel: z[p] = sum_c a[p][c] w[c] + b, fp32 sums of the exact bf16
// products in channel order; one pixel per thread, C a multiple of 8 and at most 256, rows of stride lda
__global__ __launch_bounds__(256) void head_fwd(const uint16_t* __restrict__ a, int lda, int64_t P, int C,
                                                const uint16_t* __restrict__ w, const float* __restrict__ bias,
                                                float* __restrict__ z) {
  __shared__ float ws[256];
  for (int e = threadIdx.x; e < C; e += 256) ws[e] = bf2f(w[e]);
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  float acc = 0.f;
  for (int c = 0; c < C; c += 8) {
    const uint4 v = *(const uint4*)(a + p * lda + c);
#pragma unroll
    for (int e = 0; e < 8; ++e) acc = fmaf(bf2f(u4_get(v, e)), ws[c + e], acc);
  }
  z[p] = acc + bias[0];
}

inline bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }
inline bool fits8(int64_t groups) { return groups < (int64_t(1) << 31) - 256; }

// head: y = relu(z) (the prediction); the loss compares z itself with the target, so the head's relu
// never blocks the gradient: per-work-group float64 partials of (z - t)^2 and g = bf16(2 (z - t) / cnt)
__global__ __launch_bounds__(256) void mse_loss(const float* __restrict__ z, const float* __restrict__ tgt, int64_t P,
                                                float* __restrict__ y, uint16_t* __restrict__ g,
                                                double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  const float inv = 2.0f / float(P);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < P; i += (int64_t)gridDim.x * 256) {
    const float zv = z[i], d = zv - tgt[i];
    if (y) y[i] = fmaxf(zv, 0.f);
    if (g) g[i] = f2bf(d * inv);
    acc += double(d) * double(d);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void sum_part_f64(const double* __restrict__ part, int n, int64_t P, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  out[0] = s / double(P);
}

// head input gradient: da[p][c] = g[p] * w[c] (bf16 operands, exact in fp32)
__global__ void head_dx(const uint16_t* __restrict__ g, const uint16_t* __restrict__ w, int64_t P, int C,
                        float* __restrict__ da) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= P * C) return;
  const int64_t p = t / C;
  const int c = int(t - p * C);
  da[t] = bf2f(g[p]) * bf2f(w[c]);
}

// Adam on flat fp32 arrays
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                            float bc2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ---- weight operands from the fp32 master (oracle layouts: conv W[co][ci][ky][kx], tconv W[ci][co][dy][dx])

// conv forward operand wf[co][(ky*3+kx)*Ci + ci] (Kp columns) and backward-data operand
// wd[ci][(a*3+b)*Co + co] = W[co][ci][2-a][2-b] (Kpd columns); zero padding
__global__ void prep_conv(const float* __restrict__ W, int Co, int Ci, int Kp, int Kpd, uint16_t* __restrict__ wf,
                          uint16_t* __restrict__ wd) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nf = (int64_t)Co * Kp, nd = (int64_t)Ci * Kpd;
  if (t < nf) {
    const int co = int(t / Kp), k = int(t - (int64_t)co * Kp);
    uint16_t v = 0;
    if (k < 9 * Ci) {
      const int tap = k / Ci, ci = k - tap * Ci;
      v = f2bf(W[((int64_t)co * Ci + ci) * 9 + tap]);
    }
    wf[t] = v;
  } else if (t < nf + nd) {
    const int64_t u = t - nf;
    const int ci = int(u / Kpd), k = int(u - (int64_t)ci * Kpd);
    uint16_t v = 0;
    if (k < 9 * Co) {
      const int tap = k / Co, co = k - tap * Co;
      v = f2bf(W[((int64_t)co * Ci + ci) * 9 + (8 - tap)]);
    }
    wd[u] = v;
  }
}

// transposed conv: forward operand wt[(dy*2+dx)*Co + co][ci], backward-data operand wtd[ci][(dy*2+dx)*Co + co]
__global__ void prep_tconv(const float* __restrict__ W, int Ci, int Co, uint16_t* __restrict__ wt,
                           uint16_t* __restrict__ wtd) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)Ci * Co * 4;
  if (t >= n) return;
  const int q = int(t & 3);
  const int64_t r = t >> 2;
  const int co = int(r % Co), ci = int(r / Co);
  const uint16_t v = f2bf(W[t]);   // W[ci][co][dy][dx], q = dy*2 + dx
  wt[((int64_t)q * Co + co) * Ci + ci] = v;
  wtd[(int64_t)ci * 4 * Co + q * Co + co] = v;
}

// conv gradient scatter: dWg[co][(ky*3+kx)*Ci + ci] -> dW[co][ci][ky][kx]; dWg[co][Kp] -> db[co]
__global__ void scatter_conv_grad(const float* __restrict__ dWg, int Co, int Ci, int Kp, float* __restrict__ dW,
                                  float* __restrict__ db) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)Co * Ci * 9;
  if (t < n) {
    const int tap = int(t % 9);
    const int64_t r = t / 9;
    const int ci = int(r % Ci), co = int(r / Ci);
    dW[t] = dWg[(int64_t)co * (Kp + 1) + tap * Ci + ci];
  } else if (t < n + Co) {
    const int co = int(t - n);
    db[co] = dWg[(int64_t)co * (Kp + 1) + Kp];
  }
}

// transposed-conv gradient scatter: dWg[(q*Co + co)][ci] (ld Ci+1) -> dW[ci][co][q]; db[co] = sum_q dWg[q*Co+co][Ci]
__global__ void scatter_tconv_grad(const float* __restrict__ dWg, int Ci, int Co, float* __restrict__ dW,
                                   float* __restrict__ db) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)Ci * Co * 4;
  if (t < n) {
    const int q = int(t & 3);
    const int64_t r = t >> 2;
    const int co = int(r % Co), ci = int(r / Co);
    dW[t] = dWg[((int64_t)q * Co + co) * (Ci + 1) + ci];
  } else if (t < n + Co) {
    const int co = int(t - n);
    float s = 0.f;
    for (int q = 0; q < 4; ++q) s += dWg[((int64_t)q * Co + co) * (Ci + 1) + Ci];
    db[co] = s;
  }
}

}  // namespace

// ---------------------------------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------------------------------

namespace {

enum Kind { CONV3 = 0, TCONV = 1, HEAD = 2 };

struct Layer {
  int kind, cin, cout;
  int64_t w_off, b_off;    // offsets into the flat fp32 parameter array
  int64_t op_f, op_d;      // offsets of the bf16 forward / backward-data operands
  int Kp, Kpd;             // padded contraction lengths (conv3)
};

struct Acts {              // activations of one (B, H, W), allocated on first use
  int B = 0, H = 0, W = 0;
  std::vector<sh::DevBuf<uint16_t>> enc;    // 2 per level: a, b outputs (P_l x c_l)
  std::vector<sh::DevBuf<uint16_t>> pooled; // level l >= 2 input (P_l x c_{l-1})
  std::vector<sh::DevBuf<uint8_t>> pidx;
  std::vector<sh::DevBuf<uint16_t>> cat;    // decoder level l: [tconv out, enc_l b] (P_l x 2c_l)
  std::vector<sh::DevBuf<uint16_t>> dec;    // 2 per decoder level
  sh::DevBuf<uint16_t> x0;                  // input, bf16
  sh::DevBuf<float> z;                      // head pre-activation
  // scratch
  sh::DevBuf<uint16_t> gm, gG;
  sh::DevBuf<float> f32a, gA, gB, gC, part;
  std::vector<sh::DevBuf<float>> skipg;     // decoder level l: gradient at the skip half of its concat
  sh::DevBuf<double> lpart, loss;
  sh::DevBuf<uint16_t> gbf;                 // head gradient
};

}  // namespace

struct sh_unet_s {
  int base = 0, levels = 0;
  std::vector<Layer> layers;
  int64_t nparams = 0, nops = 0;
  sh::DevBuf<float> params, grads, m, v;
  sh::DevBuf<uint16_t> ops;
  bool ops_current = false;  // ops hold the bfloat16 operands of the current params (enqueued)
  int64_t t = 0;           // Adam steps taken
  std::unique_ptr<Acts> ap;  // activations and scratch of the last (B, H, W)
  sh::DevBuf<float> dwg;     // weight-gradient product (sized at creation)
};

namespace {

int64_t P_of(const sh_unet_s* u, int l) { return (int64_t)u->ap->B * (u->ap->H >> l) * (u->ap->W >> l); }  // level l+1

sh_status ensure_acts(sh_unet u, int B, int H, int W) {
  if (u->ap && u->ap->B == B && u->ap->H == H && u->ap->W == W) return SH_OK;
  u->ap.reset();
  u->ap.reset(new (std::nothrow) Acts());
  if (!u->ap) {
    sh::set_error("host allocation failed");
    return SH_ENOMEM;
  }
  Acts& a = *u->ap;
  a.B = B;
  a.H = H;
  a.W = W;
  const int L = u->levels;
  a.enc.resize(2 * L);
  a.pooled.resize(L);
  a.pidx.resize(L);
  a.cat.resize(L);
  a.dec.resize(2 * L);
  int64_t maxf = 0, maxpart = 0;
  for (int l = 0; l < L; ++l) {
    const int64_t P = P_of(u, l);
    const int c = u->base << l;
    SH_TRY(a.enc[2 * l].alloc(P * c));
    SH_TRY(a.enc[2 * l + 1].alloc(P * c));
    if (l > 0) {
      SH_TRY(a.pooled[l].alloc(P * (c / 2)));
      SH_TRY(a.pidx[l].alloc(P * (c / 2)));
    }
    if (l < L - 1) {
      SH_TRY(a.cat[l].alloc(P * 2 * c));
      SH_TRY(a.dec[2 * l].alloc(P * c));
      SH_TRY(a.dec[2 * l + 1].alloc(P * c));
    }
    maxf = std::max(maxf, P * 4 * c);          // fp32 layer gradients / tconv outputs (<= 4c per pixel)
    maxpart = std::max(maxpart, (int64_t)8 * 1024 * 1024);
  }
  const int64_t P1 = P_of(u, 0);
  SH_TRY(a.x0.alloc(P1));
  SH_TRY(a.z.alloc(P1));
  SH_TRY(a.gbf.alloc(P1));
  SH_TRY(a.gm.alloc(maxf));
  SH_TRY(a.gG.alloc(maxf));
  SH_TRY(a.f32a.alloc(maxf));
  SH_TRY(a.gA.alloc(maxf));
  SH_TRY(a.gB.alloc(maxf));
  SH_TRY(a.gC.alloc(maxf));
  a.skipg.resize(L);
  for (int l = 0; l < L - 1; ++l) SH_TRY(a.skipg[l].alloc(P_of(u, l) * (u->base << l)));
  SH_TRY(a.part.alloc(maxpart));
  SH_TRY(a.lpart.alloc(512));
  SH_TRY(a.loss.alloc(1));
  return SH_OK;
}

// C (M x N, fp32 and/or bf16) = A (M x K) . B (N x K)^T; K % 16 == 0.  Split-K over pixels for the
// weight gradients, reduced in fixed order through `part`.
sh_status gemm(sh_unet u, const uint16_t* A, int lda, const uint16_t* B, int ldb, int64_t M, int N, int64_t K,
               const float* bias, bool relu, float* C, int ldc, uint16_t* Cb, int ldcb, bool allow_split,
               hipStream_t st, const Im2col* gat = nullptr, const Tconv* tco = nullptr, uint16_t* Cb2 = nullptr,
               int ldcb2 = 0, uint16_t* pool_out = nullptr, uint8_t* pool_idx = nullptr, bool* pooled = nullptr) {
  if (pooled) *pooled = false;
  SH_REQUIRE(K % 16 == 0 && K > 0, "internal: GEMM K = %lld not a multiple of 16", (long long)K);
  SH_REQUIRE(M < (int64_t(1) << 31) / 128, "internal: GEMM M too large");
  // products with at most 32 columns take the 128 x 32 tile, the others 64 x 64
  const bool narrow = N <= 32;
  const int TM = narrow ? 128 : 64, TN = narrow ? 32 : 64;
  const unsigned gx = (unsigned)sh::cdiv(N, TN), gy = (unsigned)sh::cdiv(M, TM);
  int S = 1;
  if (allow_split) {
    const int64_t tiles = (int64_t)gx * gy;
    S = (int)std::max<int64_t>(1, std::min<int64_t>(512 / std::max<int64_t>(tiles, 1), K / 256));
    while (S > 1 && (int64_t)S * M * N > u->ap->part.count) --S;
  }
  const int64_t kchunk = rup(sh::cdiv(K, S), GBK);
  S = (int)sh::cdiv(K, kchunk);
  const Im2col g0{nullptr, 0, 1, 1, 1};
  const Tconv tc0{nullptr, 0, 1, 1, 1}, tc = tco ? *tco : tc0;
  SH_REQUIRE(!tco || (!gat && S == 1 && !C && !Cb && !relu && bias && tco->dst && tco->Co % 8 == 0 &&
                      tco->ld % 8 == 0 && (reinterpret_cast<uintptr_t>(tco->dst) & 15) == 0 &&
                      M == (int64_t)u->ap->B * tco->h * tco->w && N == 4 * tco->Co),
             "internal: transposed-convolution output");
  SH_REQUIRE(!Cb2 || (Cb && S == 1), "internal: second output");
  if (gat && gat->C % 32 == 0 && gat->ldx % 8 == 0 && ldb % 8 == 0 && K == 9 * gat->C &&
      M * gat->ldx < (int64_t(1) << 30) && (int64_t)N * ldb < (int64_t(1) << 30) &&
      (reinterpret_cast<uintptr_t>(gat->x) & 15) == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0) {
    // direct convolution: pixel tiles of one image, output-channel tiles
    SH_REQUIRE(M == (int64_t)u->ap->B * gat->H * gat->W, "internal: convolution shape");
    const int tiles_x = (int)sh::cdiv(gat->W, 32), tiles_img = tiles_x * (int)sh::cdiv(gat->H, 8);
    // 32-channel tiles also where 64-channel tiles would leave fewer than two work-groups per CU (the deep
    // levels' small images): twice the work-groups, and the 32-channel tile's smaller LDS fits three per CU
    const bool n32 = narrow || (int64_t)tiles_img * u->ap->B * sh::cdiv(N, 64) < 512;
    const dim3 grid((unsigned)(tiles_img * u->ap->B), (unsigned)sh::cdiv(N, n32 ? 32 : 64));
    const bool staged = !C && Cb && N % 8 == 0 && ldcb % 8 == 0 && al16(Cb) && (!Cb2 || (ldcb2 % 8 == 0 && al16(Cb2)));
    const bool pool = staged && pool_out && gat->H % 2 == 0 && gat->W % 2 == 0 && al16(pool_out) &&
                      (reinterpret_cast<uintptr_t>(pool_idx) & 7) == 0;
    if (pooled) *pooled = pool;
    if (n32)
      hipLaunchKernelGGL((conv3_nt<32>), grid, dim3(256), 0, st, gat->x, gat->ldx, gat->H, gat->W, gat->C, B, ldb, N,
                         tiles_x, tiles_img, bias, relu ? 1 : 0, C, ldc, Cb, ldcb, Cb2, ldcb2, staged ? 1 : 0,
                         pool ? pool_out : nullptr, pool ? pool_idx : nullptr);
    else
      hipLaunchKernelGGL((conv3_nt<64>), grid, dim3(256), 0, st, gat->x, gat->ldx, gat->H, gat->W, gat->C, B, ldb, N,
                         tiles_x, tiles_img, bias, relu ? 1 : 0, C, ldc, Cb, ldcb, Cb2, ldcb2, staged ? 1 : 0,
                         pool ? pool_out : nullptr, pool ? pool_idx : nullptr);
  } else if (gat) {
    SH_REQUIRE(S == 1 && M == (int64_t)u->ap->B * gat->H * gat->W && K == rup(9 * gat->C, 16),
               "internal: implicit im2col shape");
    if (narrow)
      hipLaunchKernelGGL((gemm_nt<true, 1>), dim3(gx, gy, 1), dim3(256), 0, st, nullptr, 0, B, ldb, (int)M, N, (int)K,
                         (int)kchunk, bias, relu ? 1 : 0, C, ldc, Cb, ldcb, *gat, tc0, Cb2, ldcb2);
    else
      hipLaunchKernelGGL((gemm_nt<true, 2>), dim3(gx, gy, 1), dim3(256), 0, st, nullptr, 0, B, ldb, (int)M, N, (int)K,
                         (int)kchunk, bias, relu ? 1 : 0, C, ldc, Cb, ldcb, *gat, tc0, Cb2, ldcb2);
  } else if (S == 1) {
    if (narrow)
      hipLaunchKernelGGL((gemm_nt<false, 1>), dim3(gx, gy, 1), dim3(256), 0, st, A, lda, B, ldb, (int)M, N, (int)K,
                         (int)kchunk, bias, relu ? 1 : 0, C, ldc, Cb, ldcb, g0, tc, Cb2, ldcb2);
    else
      hipLaunchKernelGGL((gemm_nt<false, 2>), dim3(gx, gy, 1), dim3(256), 0, st, A, lda, B, ldb, (int)M, N, (int)K,
                         (int)kchunk, bias, relu ? 1 : 0, C, ldc, Cb, ldcb, g0, tc, Cb2, ldcb2);
  } else {
    SH_REQUIRE(C && !Cb && !bias && !relu && ldc == N, "internal: split GEMM writes plain fp32");
    if (narrow)
      hipLaunchKernelGGL((gemm_nt<false, 1>), dim3(gx, gy, S), dim3(256), 0, st, A, lda, B, ldb, (int)M, N, (int)K,
                         (int)kchunk, nullptr, 0, u->ap->part.ptr, N, nullptr, 0, g0, tc0, nullptr, 0);
    else
      hipLaunchKernelGGL((gemm_nt<false, 2>), dim3(gx, gy, S), dim3(256), 0, st, A, lda, B, ldb, (int)M, N, (int)K,
                         (int)kchunk, nullptr, 0, u->ap->part.ptr, N, nullptr, 0, g0, tc0, nullptr, 0);
    hipLaunchKernelGGL(sum_splits, dim3(nb(M * N)), dim3(256), 0, st, u->ap->part.ptr, S, M * N, C);
  }
  SH_LAUNCHED();
  return SH_OK;
}

// Weight gradient C (M x (NB + ones), fp32, row stride NB + ones) = sum over P pixels of A[p]^T Bv[p]
// (gemm_tn), split over pixels and reduced in fixed order through `part` when the tile grid is small.
sh_status gemm_wgrad(sh_unet u, const uint16_t* A, int lda, int M, const uint16_t* B, int ldb, int NB, bool ones,
                     int64_t P, float* C, hipStream_t st, const Im2col* gat = nullptr) {
  SH_REQUIRE(NB % 8 == 0 && P > 0 && P < (int64_t(1) << 31), "internal: weight-gradient shape");
  const int N = NB + (ones ? 1 : 0);
  const unsigned gx = (unsigned)sh::cdiv(N, GBN), gy = (unsigned)sh::cdiv(M, GBM);
  const int64_t tiles = (int64_t)gx * gy;
  int S = (int)std::max<int64_t>(1, std::min<int64_t>(512 / std::max<int64_t>(tiles, 1), P / 256));
  while (S > 1 && (int64_t)S * M * N > u->ap->part.count) --S;
  const int64_t kchunk = rup(sh::cdiv(P, S), GBK);
  S = (int)sh::cdiv(P, kchunk);
  if (gat && ones && gat->C % 32 == 0 && M % 32 == 0 && NB == 9 * gat->C && lda % 8 == 0 && gat->ldx % 8 == 0 &&
      al16(A) && al16(gat->x) && P == (int64_t)u->ap->B * gat->H * gat->W) {
    // direct form: pixel tiles of 8 x 32 split over the work-groups, partials in the same layout
    const int tiles_x = (int)sh::cdiv(gat->W, 32), tiles_img = tiles_x * (int)sh::cdiv(gat->H, 8);
    const int ntiles = tiles_img * u->ap->B;
    const int blocks = (gat->C / 32) * (M / 32);
    int Sd = (int)std::max<int64_t>(1, std::min<int64_t>(256 / blocks, ntiles));
    while (Sd > 1 && (int64_t)Sd * M * N > u->ap->part.count) --Sd;
    const int per = (int)sh::cdiv(ntiles, Sd);
    Sd = (int)sh::cdiv(ntiles, per);
    float* dstd = Sd == 1 ? C : u->ap->part.ptr;
    hipLaunchKernelGGL(wgrad3, dim3(gat->C / 32, M / 32, Sd), dim3(256), 0, st, A, lda, gat->x, gat->ldx, gat->H,
                       gat->W, gat->C, M, tiles_x, tiles_img, ntiles, per, dstd);
    if (Sd > 1) hipLaunchKernelGGL(sum_splits, dim3(nb((int64_t)M * N)), dim3(256), 0, st, u->ap->part.ptr, Sd,
                                   (int64_t)M * N, C);
    SH_LAUNCHED();
    return SH_OK;
  }
  const Im2col g = gat ? *gat : Im2col{nullptr, 0, 1, 1, 1};
  float* dst = S == 1 ? C : u->ap->part.ptr;
  if (gat)
    hipLaunchKernelGGL(gemm_tn<true>, dim3(gx, gy, S), dim3(256), 0, st, A, lda, M, nullptr, 0, NB, ones ? 1 : 0, N,
                       (int)P, (int)kchunk, dst, N, g);
  else
    hipLaunchKernelGGL(gemm_tn<false>, dim3(gx, gy, S), dim3(256), 0, st, A, lda, M, B, ldb, NB, ones ? 1 : 0, N,
                       (int)P, (int)kchunk, dst, N, g);
  if (S > 1) hipLaunchKernelGGL(sum_splits, dim3(nb((int64_t)M * N)), dim3(256), 0, st, u->ap->part.ptr, S,
                                (int64_t)M * N, C);
  SH_LAUNCHED();
  return SH_OK;
}

// The products' bfloat16 weight operands from the float32 parameters, again only after the parameters changed
// (set_params, an Adam step): repeated forward passes with the same weights reuse them.  The conversion is
// enqueued on st, ahead of the products that read it on the same stream.
sh_status prep_weights(sh_unet u, hipStream_t st) {
  if (u->ops_current) return SH_OK;
  for (const Layer& ly : u->layers) {
    const float* W = u->params.ptr + ly.w_off;
    uint16_t* of = u->ops.ptr + ly.op_f;
    uint16_t* od = u->ops.ptr + ly.op_d;
    if (ly.kind == CONV3) {
      const int64_t n = (int64_t)ly.cout * ly.Kp + (int64_t)ly.cin * ly.Kpd;
      hipLaunchKernelGGL(prep_conv, dim3(nb(n)), dim3(256), 0, st, W, ly.cout, ly.cin, ly.Kp, ly.Kpd, of, od);
    } else if (ly.kind == TCONV) {
      hipLaunchKernelGGL(prep_tconv, dim3(nb((int64_t)ly.cin * ly.cout * 4)), dim3(256), 0, st, W, ly.cin, ly.cout, of,
                         od);
    } else {
      hipLaunchKernelGGL(f32_to_bf16, dim3(nb(ly.cin)), dim3(256), 0, st, W, of, (int64_t)ly.cin);
    }
  }
  SH_LAUNCHED();
  u->ops_current = true;
  return SH_OK;
}

// conv3 forward: out (P x Co, bf16) = relu(im2col(in) . wf^T + b)
sh_status conv_fwd(sh_unet u, const Layer& ly, const uint16_t* in, int ldin, int B, int H, int W, uint16_t* out,
                   hipStream_t st, uint16_t* out2 = nullptr, int ld2 = 0, uint16_t* pool_out = nullptr,
                   uint8_t* pool_idx = nullptr, bool* pooled = nullptr) {
  if (pooled) *pooled = false;
  const int64_t P = (int64_t)B * H * W;
  if (ly.cin == 1 && ly.cout % 8 == 0 && ly.cout <= 64 && fits8(P) && al16(out) && !out2) {   // the first layer
    hipLaunchKernelGGL(conv3_c1, dim3(nb(P)), dim3(256), 0, st, in, ldin, B, H, W, u->ops.ptr + ly.op_f, ly.Kp,
                       ly.cout, u->params.ptr + ly.b_off, out, ly.cout);
    SH_LAUNCHED();
    return SH_OK;
  }
  const Im2col g{in, ldin, H, W, ly.cin};
  return gemm(u, nullptr, 0, u->ops.ptr + ly.op_f, ly.Kp, P, ly.cout, ly.Kp, u->params.ptr + ly.b_off, true, nullptr, 0,
              out, ly.cout, false, st, &g, nullptr, out2, ld2, pool_out, pool_idx, pooled);
}

// conv3 backward.  gin (+ gin2, strided) is the fp32 gradient at the layer's post-ReLU output `out`.
// Writes the weight and bias gradients and, if dx is set, the fp32 gradient at the input.
sh_status conv_bwd(sh_unet u, const Layer& ly, const uint16_t* in, int ldin, const uint16_t* out, const float* gin,
                   int ldg, const float* gin2, int ldg2, int B, int H, int W, float* dx, hipStream_t st) {
  Acts& a = *u->ap;
  const int64_t P = (int64_t)B * H * W;
  if (ly.cout % 8 == 0 && ldg % 4 == 0 && (!gin2 || ldg2 % 4 == 0) && al16(gin) && (!gin2 || al16(gin2)) &&
      fits8(P * ly.cout / 8))
    hipLaunchKernelGGL(relu_mask_grad8, dim3(nb(P * ly.cout / 8)), dim3(256), 0, st, gin, ldg, gin2, ldg2, out, (int)P,
                       ly.cout, a.gm.ptr);
  else
    hipLaunchKernelGGL(relu_mask_grad, dim3(nb(P * ly.cout)), dim3(256), 0, st, gin, ldg, gin2, ldg2, out, P, ly.cout,
                       a.gm.ptr);
  // weight gradient: dWg[co][k] = sum_p gm[p][co] [im2col(in), 1][p][k] (k = Kp: the bias)
  const Im2col gi{in, ldin, H, W, ly.cin};
  SH_TRY(gemm_wgrad(u, a.gm.ptr, ly.cout, ly.cout, nullptr, 0, ly.Kp, true, P, u->dwg.ptr, st, &gi));
  const int64_t ns = (int64_t)ly.cout * ly.cin * 9 + ly.cout;
  hipLaunchKernelGGL(scatter_conv_grad, dim3(nb(ns)), dim3(256), 0, st, u->dwg.ptr, ly.cout, ly.cin, ly.Kp,
                     u->grads.ptr + ly.w_off, u->grads.ptr + ly.b_off);
  SH_LAUNCHED();
  if (!dx) return SH_OK;
  // input gradient: im2col(gm) . wd^T, im2col implicit
  const Im2col g{a.gm.ptr, ly.cout, H, W, ly.cout};
  return gemm(u, nullptr, 0, u->ops.ptr + ly.op_d, ly.Kpd, P, ly.cin, ly.Kpd, nullptr, false, dx, ly.cin, nullptr, 0,
              false, st, &g);
}

// Forward pass over B images of H x W (input x fp32 device), keeping every activation.
sh_status net_forward(sh_unet u, const float* x, int B, int H, int W, hipStream_t st) {
  SH_TRY(ensure_acts(u, B, H, W));
  SH_TRY(prep_weights(u, st));
  Acts& a = *u->ap;
  const int L = u->levels;
  const int64_t P1 = (int64_t)B * H * W;
  hipLaunchKernelGGL(f32_to_bf16, dim3(nb(P1)), dim3(256), 0, st, x, a.x0.ptr, P1);
  const uint16_t* cur = a.x0.ptr;
  int ldc = 1;
  int li = 0;
  bool pooled = false;   // the previous level's convolution also wrote this level's pooled input
  for (int l = 0; l < L; ++l) {
    const int h = H >> l, w = W >> l, c = u->base << l;
    if (l > 0) {
      const int pc = c / 2;
      if (!pooled) {
        if (pc % 8 == 0 && fits8((int64_t)B * h * w * pc / 8))
          hipLaunchKernelGGL(pool_fwd8, dim3(nb((int64_t)B * h * w * pc / 8)), dim3(256), 0, st, a.enc[2 * l - 1].ptr,
                             B, 2 * h, 2 * w, pc, a.pooled[l].ptr, a.pidx[l].ptr);
        else
          hipLaunchKernelGGL(pool_fwd, dim3(nb((int64_t)B * h * w * pc)), dim3(256), 0, st, a.enc[2 * l - 1].ptr, B,
                             2 * h, 2 * w, pc, a.pooled[l].ptr, a.pidx[l].ptr);
      }
      cur = a.pooled[l].ptr;
      ldc = pc;
    }
    SH_TRY(conv_fwd(u, u->layers[li++], cur, ldc, B, h, w, a.enc[2 * l].ptr, st));
    // below the bottleneck the output is also the skip half of the decoder's concatenation (channels c..2c-1)
    // and the next level's pooled input, when the convolution can form it
    uint16_t* skip = l < L - 1 ? a.cat[l].ptr + c : nullptr;
    SH_TRY(conv_fwd(u, u->layers[li++], a.enc[2 * l].ptr, c, B, h, w, a.enc[2 * l + 1].ptr, st, skip, 2 * c,
                    l < L - 1 ? a.pooled[l + 1].ptr : nullptr, l < L - 1 ? a.pidx[l + 1].ptr : nullptr, &pooled));
    cur = a.enc[2 * l + 1].ptr;
    ldc = c;
  }
  for (int l = L - 2; l >= 0; --l) {
    const int h = H >> l, w = W >> l, c = u->base << l;
    const int64_t Pin = (int64_t)B * (h / 2) * (w / 2), P = (int64_t)B * h * w;
    const Layer& tl = u->layers[li++];
    if (c % 8 == 0 && fits8(P * c / 8)) {
      // the upsampled half of the concatenation straight from the product's epilogue
      const Tconv tcv{a.cat[l].ptr, 2 * c, h / 2, w / 2, c};
      SH_TRY(gemm(u, cur, ldc, u->ops.ptr + tl.op_f, tl.cin, Pin, 4 * c, tl.cin, u->params.ptr + tl.b_off, false,
                  nullptr, 0, nullptr, 0, false, st, nullptr, &tcv));
    } else {
      SH_TRY(gemm(u, cur, ldc, u->ops.ptr + tl.op_f, tl.cin, Pin, 4 * c, tl.cin, nullptr, false, a.f32a.ptr, 4 * c,
                  nullptr, 0, false, st));
      hipLaunchKernelGGL(tconv_scatter, dim3(nb(Pin * 4 * c)), dim3(256), 0, st, a.f32a.ptr, u->params.ptr + tl.b_off,
                         B, h / 2, w / 2, c, a.cat[l].ptr, 2 * c);
    }
    SH_TRY(conv_fwd(u, u->layers[li++], a.cat[l].ptr, 2 * c, B, h, w, a.dec[2 * l].ptr, st));
    SH_TRY(conv_fwd(u, u->layers[li++], a.dec[2 * l].ptr, c, B, h, w, a.dec[2 * l + 1].ptr, st));
    cur = a.dec[2 * l + 1].ptr;
    ldc = c;
  }
  const Layer& hd = u->layers[li];
  if (hd.cin % 8 == 0 && hd.cin <= 256 && ldc % 8 == 0 && al16(cur)) {
    hipLaunchKernelGGL(head_fwd, dim3(nb(P1)), dim3(256), 0, st, cur, ldc, P1, hd.cin, u->ops.ptr + hd.op_f,
                       u->params.ptr + hd.b_off, a.z.ptr);
    SH_LAUNCHED();
    return SH_OK;
  }
  return gemm(u, cur, ldc, u->ops.ptr + hd.op_f, hd.cin, P1, 1, hd.cin, u->params.ptr + hd.b_off, false, a.z.ptr, 1,
              nullptr, 0, false, st);
}

// fp32 strided copy: dst[p*C + c] = src[p*lds + off + c]
__global__ void copy_f32_channels(const float* __restrict__ src, int lds, int off, float* __restrict__ dst, int64_t P,
                                  int C) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= P * C) return;
  const int64_t p = t / C;
  const int c = int(t - p * C);
  dst[t] = src[p * lds + off + c];
}

// the same, four channels per thread (C, lds and off multiples of 4, 16-byte aligned buffers)
__global__ void copy_f32_channels4(const float* __restrict__ src, int lds, int off, float* __restrict__ dst, int P,
                                   int C) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int C4 = C >> 2;
  if (t >= P * C4) return;
  const int p = t / C4, c = 4 * (t - p * C4);
  *(float4*)(dst + 4 * (int64_t)t) = *(const float4*)(src + (int64_t)p * lds + off + c);
}

// Backward pass after net_forward (every parameter gradient into u->grads); target fp32 device.
// The loss lands in a.loss (device) and relu(z) in y_out if given.
sh_status net_backward(sh_unet u, const float* target, float* y_out, hipStream_t st) {
  Acts& a = *u->ap;
  const int B = a.B, H = a.H, W = a.W, L = u->levels;
  const int64_t P1 = (int64_t)B * H * W;
  const int nblocks = 256;
  hipLaunchKernelGGL(mse_loss, dim3(nblocks), dim3(256), 0, st, a.z.ptr, target, P1, y_out, a.gbf.ptr, a.lpart.ptr);
  hipLaunchKernelGGL(sum_part_f64, dim3(1), dim3(64), 0, st, a.lpart.ptr, nblocks, P1, a.loss.ptr);
  const int nl = (int)u->layers.size();
  // head: dW = g^T . [a^T; 1]^T, da = g w
  const Layer& hd = u->layers[nl - 1];
  const uint16_t* hin = L > 1 ? a.dec[1].ptr : a.enc[1].ptr;
  const int c1 = u->base;
  SH_TRY(gemm_wgrad(u, a.gbf.ptr, 1, 1, hin, c1, c1, true, P1, u->dwg.ptr, st));
  hipLaunchKernelGGL(copy_f32_channels, dim3(1), dim3(256), 0, st, u->dwg.ptr, c1 + 1, 0, u->grads.ptr + hd.w_off,
                     (int64_t)1, c1);
  hipLaunchKernelGGL(copy_f32_channels, dim3(1), dim3(256), 0, st, u->dwg.ptr, c1 + 1, c1, u->grads.ptr + hd.b_off,
                     (int64_t)1, 1);
  hipLaunchKernelGGL(head_dx, dim3(nb(P1 * c1)), dim3(256), 0, st, a.gbf.ptr, u->ops.ptr + hd.op_f, P1, c1, a.gA.ptr);
  SH_LAUNCHED();
  // decoder, level 1 first; gA holds the gradient at the current level's last output
  int li = nl - 2;
  for (int l = 0; l < L - 1; ++l) {
    const int h = H >> l, w = W >> l, c = u->base << l;
    const int64_t P = (int64_t)B * h * w, Pin = (int64_t)B * (h / 2) * (w / 2);
    const Layer& lb = u->layers[li--];
    const Layer& la = u->layers[li--];
    const Layer& tl = u->layers[li--];
    SH_TRY(conv_bwd(u, lb, a.dec[2 * l].ptr, c, a.dec[2 * l + 1].ptr, a.gA.ptr, c, nullptr, 0, B, h, w, a.gB.ptr, st));
    SH_TRY(conv_bwd(u, la, a.cat[l].ptr, 2 * c, a.dec[2 * l].ptr, a.gB.ptr, c, nullptr, 0, B, h, w, a.gC.ptr, st));
    // gC = gradient at [upsampled, skip]; the skip half waits for encoder level l
    if (c % 4 == 0 && fits8(P * c / 4))
      hipLaunchKernelGGL(copy_f32_channels4, dim3(nb(P * c / 4)), dim3(256), 0, st, a.gC.ptr, 2 * c, c,
                         a.skipg[l].ptr, (int)P, c);
    else
      hipLaunchKernelGGL(copy_f32_channels, dim3(nb(P * c)), dim3(256), 0, st, a.gC.ptr, 2 * c, c, a.skipg[l].ptr, P,
                         c);
    // transposed convolution from the upsampled half
    const int cin = tl.cin;
    const uint16_t* tin = l + 1 < L - 1 ? a.dec[2 * (l + 1) + 1].ptr : a.enc[2 * (l + 1) + 1].ptr;
    if (c % 8 == 0 && fits8(Pin * c / 2))
      hipLaunchKernelGGL(tconv_gather8, dim3(nb(Pin * c / 2)), dim3(256), 0, st, a.gC.ptr, 2 * c, B, h / 2, w / 2, c,
                         a.gG.ptr);
    else
      hipLaunchKernelGGL(tconv_gather, dim3(nb(Pin * 4 * c)), dim3(256), 0, st, a.gC.ptr, 2 * c, B, h / 2, w / 2, c,
                         a.gG.ptr);
    SH_TRY(gemm_wgrad(u, a.gG.ptr, 4 * c, 4 * c, tin, cin, cin, true, Pin, u->dwg.ptr, st));
    hipLaunchKernelGGL(scatter_tconv_grad, dim3(nb((int64_t)cin * c * 4 + c)), dim3(256), 0, st, u->dwg.ptr, cin, c,
                       u->grads.ptr + tl.w_off, u->grads.ptr + tl.b_off);
    SH_LAUNCHED();
    SH_TRY(gemm(u, a.gG.ptr, 4 * c, u->ops.ptr + tl.op_d, 4 * c, Pin, cin, 4 * c, nullptr, false, a.gA.ptr, cin,
                nullptr, 0, false, st));
  }
  // encoder, bottleneck first
  for (int l = L - 1; l >= 0; --l) {
    const int h = H >> l, w = W >> l, c = u->base << l;
    const Layer& lb = u->layers[2 * l + 1];
    const Layer& la = u->layers[2 * l];
    const float* skip = l < L - 1 ? a.skipg[l].ptr : nullptr;
    SH_TRY(conv_bwd(u, lb, a.enc[2 * l].ptr, c, a.enc[2 * l + 1].ptr, a.gA.ptr, c, skip, c, B, h, w, a.gB.ptr, st));
    const uint16_t* in = l > 0 ? a.pooled[l].ptr : a.x0.ptr;
    const int ldin = l > 0 ? c / 2 : 1;
    SH_TRY(conv_bwd(u, la, in, ldin, a.enc[2 * l].ptr, a.gB.ptr, c, nullptr, 0, B, h, w, l > 0 ? a.gC.ptr : nullptr,
                    st));
    if (l > 0) {
      const int pc = c / 2;
      if (pc % 8 == 0 && fits8((int64_t)B * h * w * pc / 8))
        hipLaunchKernelGGL(pool_bwd8, dim3(nb((int64_t)B * h * w * pc / 8)), dim3(256), 0, st, a.gC.ptr, a.pidx[l].ptr,
                           B, 2 * h, 2 * w, pc, a.gA.ptr);
      else
        hipLaunchKernelGGL(pool_bwd, dim3(nb((int64_t)B * h * w * pc)), dim3(256), 0, st, a.gC.ptr, a.pidx[l].ptr, B,
                           2 * h, 2 * w, pc, a.gA.ptr);
      SH_LAUNCHED();
    }
  }
  return SH_OK;
}

sh_status check_shape(sh_unet u, const float* x, int B, int H, int W) {
  SH_REQUIRE(u && x, "NULL argument");
  const int m = 1 << (u->levels - 1);
  SH_REQUIRE(B >= 1 && H >= m && W >= m && H % m == 0 && W % m == 0,
             "B >= 1 and H, W divisible by 2^(levels-1) = %d required (got %d x %d x %d)", m, B, H, W);
  SH_REQUIRE((int64_t)B * H * W <= (int64_t(1) << 26), "B*H*W must be <= 2^26");
  return SH_OK;
}

}  // namespace

extern "C" {

sh_status sh_unet_create(int32_t base, int32_t levels, sh_unet* out) {
  SH_REQUIRE(out, "out is NULL");
  *out = nullptr;
  SH_REQUIRE(base >= 16 && base <= 128 && base % 16 == 0, "base channels must be a multiple of 16 in [16, 128]");
  SH_REQUIRE(levels >= 1 && levels <= 6, "levels must be in [1, 6]");
  std::unique_ptr<sh_unet_s> u(new (std::nothrow) sh_unet_s());
  if (!u) {
    sh::set_error("host allocation failed");
    return SH_ENOMEM;
  }
  u->base = base;
  u->levels = levels;
  int64_t off = 0, oo = 0, dwg = 0;
  auto add = [&](int kind, int cin, int cout) {
    Layer ly{kind, cin, cout, 0, 0, 0, 0, 0, 0};
    const int64_t nw = kind == CONV3 ? (int64_t)cout * cin * 9 : kind == TCONV ? (int64_t)cin * cout * 4 : cin;
    ly.w_off = off;
    ly.b_off = off + nw;
    off += nw + cout;
    if (kind == CONV3) {
      ly.Kp = (int)rup(9 * cin, 16);
      ly.Kpd = (int)rup(9 * cout, 16);
      ly.op_f = oo;
      ly.op_d = oo + (int64_t)cout * ly.Kp;
      oo += (int64_t)cout * ly.Kp + (int64_t)cin * ly.Kpd;
      dwg = std::max<int64_t>(dwg, (int64_t)cout * (ly.Kp + 1));
    } else if (kind == TCONV) {
      ly.op_f = oo;
      ly.op_d = oo + (int64_t)cin * cout * 4;
      oo += (int64_t)cin * cout * 8;
      dwg = std::max<int64_t>(dwg, (int64_t)4 * cout * (cin + 1));
    } else {
      ly.op_f = ly.op_d = oo;
      oo += rup(cin, 16);
      dwg = std::max<int64_t>(dwg, cin + 1);
    }
    u->layers.push_back(ly);
  };
  for (int l = 0; l < levels; ++l) {
    const int c = base << l;
    add(CONV3, l == 0 ? 1 : c / 2, c);
    add(CONV3, c, c);
  }
  for (int l = levels - 2; l >= 0; --l) {
    const int c = base << l;
    add(TCONV, 2 * c, c);
    add(CONV3, 2 * c, c);
    add(CONV3, c, c);
  }
  add(HEAD, base, 1);
  u->nparams = off;
  u->nops = oo;
  SH_TRY(u->params.alloc(off));
  SH_TRY(u->grads.alloc(off));
  SH_TRY(u->m.alloc(off));
  SH_TRY(u->v.alloc(off));
  SH_TRY(u->ops.alloc(oo));
  SH_TRY(u->dwg.alloc(dwg));
  SH_HIP(hipMemset(u->params.ptr, 0, off * sizeof(float)));
  SH_HIP(hipMemset(u->grads.ptr, 0, off * sizeof(float)));
  SH_HIP(hipMemset(u->m.ptr, 0, off * sizeof(float)));
  SH_HIP(hipMemset(u->v.ptr, 0, off * sizeof(float)));
  SH_HIP(hipMemset(u->ops.ptr, 0, oo * sizeof(uint16_t)));
  *out = u.release();
  return SH_OK;
}

sh_status sh_unet_destroy(sh_unet u) {
  delete u;
  return SH_OK;
}

sh_status sh_unet_num_params(sh_unet u, int64_t* n_out) {
  SH_REQUIRE(u && n_out, "NULL argument");
  *n_out = u->nparams;
  return SH_OK;
}

sh_status sh_unet_set_params(sh_unet u, const float* host, int64_t n) {
  SH_REQUIRE(u && host, "NULL argument");
  SH_REQUIRE(n == u->nparams, "expected %lld parameters, got %lld", (long long)u->nparams, (long long)n);
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(host[i])) {
      sh::set_error("parameter %lld is not finite", (long long)i);
      return SH_ENONFINITE;
    }
  SH_HIP(hipMemcpy(u->params.ptr, host, n * sizeof(float), hipMemcpyHostToDevice));
  u->ops_current = false;
  SH_HIP(hipMemset(u->m.ptr, 0, n * sizeof(float)));
  SH_HIP(hipMemset(u->v.ptr, 0, n * sizeof(float)));
  u->t = 0;
  return SH_OK;
}

sh_status sh_unet_get_params(sh_unet u, float* host, int64_t n) {
  SH_REQUIRE(u && host, "NULL argument");
  SH_REQUIRE(n == u->nparams, "expected %lld parameters, got %lld", (long long)u->nparams, (long long)n);
  SH_HIP(hipMemcpy(host, u->params.ptr, n * sizeof(float), hipMemcpyDeviceToHost));
  return SH_OK;
}

sh_status sh_unet_forward(sh_unet u, const float* x, int32_t B, int32_t H, int32_t W, float* y, void* stream) {
  SH_TRY(check_shape(u, x, B, H, W));
  SH_REQUIRE(y, "y is NULL");
  hipStream_t st = (hipStream_t)stream;
  SH_TRY(net_forward(u, x, B, H, W, st));
  hipLaunchKernelGGL(mse_loss, dim3(64), dim3(256), 0, st, u->ap->z.ptr, u->ap->z.ptr, (int64_t)B * H * W, y, nullptr,
                     u->ap->lpart.ptr);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status sh_unet_loss_grad(sh_unet u, const float* x, const float* target, int32_t B, int32_t H, int32_t W,
                            double* loss_out, float* grads_host, void* stream) {
  SH_TRY(check_shape(u, x, B, H, W));
  SH_REQUIRE(target && loss_out, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  SH_TRY(net_forward(u, x, B, H, W, st));
  SH_TRY(net_backward(u, target, nullptr, st));
  SH_HIP(hipMemcpyAsync(loss_out, u->ap->loss.ptr, sizeof(double), hipMemcpyDeviceToHost, st));
  if (grads_host)
    SH_HIP(hipMemcpyAsync(grads_host, u->grads.ptr, u->nparams * sizeof(float), hipMemcpyDeviceToHost, st));
  SH_HIP(hipStreamSynchronize(st));
  return SH_OK;
}

sh_status sh_unet_train_step(sh_unet u, const float* x, const float* target, int32_t B, int32_t H, int32_t W,
                             float lr, double* loss_out, void* stream) {
  SH_TRY(check_shape(u, x, B, H, W));
  SH_REQUIRE(target, "target is NULL");
  SH_REQUIRE(std::isfinite(lr) && lr > 0.f, "lr must be positive");
  hipStream_t st = (hipStream_t)stream;
  SH_TRY(net_forward(u, x, B, H, W, st));
  SH_TRY(net_backward(u, target, nullptr, st));
  u->t += 1;
  const double b1 = 0.9, b2 = 0.999;
  hipLaunchKernelGGL(adam_kernel, dim3(nb(u->nparams)), dim3(256), 0, st, u->params.ptr, u->grads.ptr, u->m.ptr,
                     u->v.ptr, u->nparams, lr, (float)b1, (float)b2, 1e-8f, (float)(1.0 - std::pow(b1, (double)u->t)),
                     (float)(1.0 - std::pow(b2, (double)u->t)));
  SH_LAUNCHED();
  u->ops_current = false;
  if (loss_out) {
    SH_HIP(hipMemcpyAsync(loss_out, u->ap->loss.ptr, sizeof(double), hipMemcpyDeviceToHost, st));
    SH_HIP(hipStreamSynchronize(st));
  }
  return SH_OK;
}

}  // extern "C"

// ---- warm start: x0 = s U(d / s), d = Phi^dagger y / PSF peak, s = RMS of d, per problem ----------------

namespace {

__global__ void delta_images(float* __restrict__ d, int n) {   // grid (cdiv(n*n, 256), P)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)n * n) return;
  d[(int64_t)blockIdx.y * n * n + i] = i == (int64_t)(n / 2) * n + n / 2 ? 1.f : 0.f;
}

// per problem (work-group p): peak = psf[p](centre); s = RMS(d_p) / peak; in = d_p / peak / s
__global__ __launch_bounds__(256) void normalise_dirty(const float* __restrict__ psf, const float* __restrict__ d,
                                                       int n, float* __restrict__ in, float* __restrict__ scale) {
  __shared__ double sm[256];
  const int64_t N = (int64_t)n * n, off = (int64_t)blockIdx.x * N;
  const float peak = psf[off + (int64_t)(n / 2) * n + n / 2];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += 256) m += double(d[off + i]) * double(d[off + i]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
    __syncthreads();
  }
  const float sc = fmaxf(float(sqrt(sm[0] / double(N))) / peak, 1e-30f);
  const float inv = 1.f / (peak * sc);
  for (int64_t i = threadIdx.x; i < N; i += 256) in[off + i] = d[off + i] * inv;
  if (threadIdx.x == 0) scale[blockIdx.x] = sc;
}

__global__ void rescale(float* __restrict__ x, const float* __restrict__ scale, int64_t N) {   // grid (.., P)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) x[(int64_t)blockIdx.y * N + i] *= scale[blockIdx.y];
}

__global__ void rescale_inv(float* __restrict__ x, const float* __restrict__ scale, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) x[(int64_t)blockIdx.y * N + i] /= scale[blockIdx.y];
}

}  // namespace

extern "C" {

sh_status sh_dirty_normalised(sh_op op, const float* y, float* d_out, float* scale_out, void* stream) {
  SH_REQUIRE(op && y && d_out && scale_out, "NULL argument");
  const int n = op->n, P = op->P;
  hipStream_t st = (hipStream_t)stream;
  const int64_t N = (int64_t)n * n;
  sh::DevBuf<float> d, psf;
  sh::DevBuf<float2> v;
  SH_TRY(d.alloc(N * P));
  SH_TRY(psf.alloc(N * P));
  SH_TRY(v.alloc(op->M));
  hipLaunchKernelGGL(delta_images, dim3(nb(N), P), dim3(256), 0, st, d.ptr, n);
  SH_LAUNCHED();
  SH_TRY(sh::phi_forward(op, d.ptr, v.ptr, false, nullptr, st));
  SH_TRY(sh::phi_adjoint(op, v.ptr, psf.ptr, false, nullptr, st));
  SH_TRY(sh::phi_adjoint(op, (const float2*)y, d.ptr, true, nullptr, st));
  hipLaunchKernelGGL(normalise_dirty, dim3(P), dim3(256), 0, st, psf.ptr, d.ptr, n, d_out, scale_out);
  SH_LAUNCHED();
  SH_HIP(hipStreamSynchronize(st));   // scratch is freed on return
  return SH_OK;
}

sh_status sh_scale_images(float* x, const float* scale, int32_t P, int64_t N, int32_t invert, void* stream) {
  SH_REQUIRE(x && scale && P >= 1 && N >= 1, "invalid argument");
  hipStream_t st = (hipStream_t)stream;
  if (invert)
    hipLaunchKernelGGL(rescale_inv, dim3(nb(N), P), dim3(256), 0, st, x, scale, N);
  else
    hipLaunchKernelGGL(rescale, dim3(nb(N), P), dim3(256), 0, st, x, scale, N);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status sh_warm_start(sh_unet u, sh_op op, const float* y, float* x0_out, void* stream) {
  SH_REQUIRE(u && op && y && x0_out, "NULL argument");
  const int n = op->n, P = op->P;
  const int m = 1 << (u->levels - 1);
  SH_REQUIRE(n % m == 0, "image side %d not divisible by 2^(levels-1) = %d", n, m);
  hipStream_t st = (hipStream_t)stream;
  const int64_t N = (int64_t)n * n;
  sh::DevBuf<float> in, sc;
  SH_TRY(in.alloc(N * P));
  SH_TRY(sc.alloc(P));
  SH_TRY(sh_dirty_normalised(op, y, in.ptr, sc.ptr, stream));
  SH_TRY(sh_unet_forward(u, in.ptr, P, n, n, x0_out, stream));
  hipLaunchKernelGGL(rescale, dim3(nb(N), P), dim3(256), 0, st, x0_out, sc.ptr, N);
  SH_LAUNCHED();
  SH_HIP(hipStreamSynchronize(st));   // scratch is freed on return
  return SH_OK;
}

}  // extern "C"
