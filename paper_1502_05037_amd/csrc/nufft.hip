// Measurement operator Phi and its real adjoint (measurement equation y = Phi x + n; block split (2)).
//
// Phi = G F Z S: the FFT passes live in fft.hip; this file holds the planner and the interpolation
// kernels G (degridding) and G^H (gridding) with a J x J Kaiser-Bessel kernel.
//
// Coordinates.  kappa = u K / (2 pi) is split on the host, in float64, into the grid cell
// floor(kappa) mod K and the fraction kappa - floor(kappa); both are packed into one uint32 per axis
// (cell in the top log2 K bits, the fraction truncated to the remaining bits), so the tap window is
// the one float64 gives and the fraction is exact in float32.
//
// Order.  Inside each data block the visibilities are sorted by (uv tile of T x T cells, cell), so
// blocks stay contiguous ("internal order": a permutation inside each block).  A work item is a
// contiguous run of internal order with one (block, tile), cut into chunks of at most GRID_CHUNK.
//
// Degridding: one work-group per item stages the tile's padded (T+J-1)^2 grid patch in LDS; its threads
// take the item's visibilities interleaved (coalesced loads and stores) and read each one's J x J window
// from LDS.
//
// Gridding (atomic-free): one work-group per item owns a private padded patch, written to the item's own
// slot; the fold kernel then forms each grid cell as the sum, in a fixed order, of the patches that cover
// it.  Every sum has a fixed order, so the adjoint is bitwise reproducible.
//  * J = 8 (grid_mfma_kernel): the outer products w1 w2^T v of a run of visibilities in one cell accumulate
//    on the matrix cores (v_mfma_f32_4x4x1_16b_f32, full fp32), two visibilities per instruction; each
//    half-wave is a stream over its share of the item with its own copy of the rows of the patch it touches.
//  * other J (grid_kernel): phase A computes the 2J one-dimensional weights of a batch of visibilities, two
//    lanes each (one per axis), into LDS.  Phase B walks the batch wave by wave with one lane per tap
//    (t1, t2): the lane accumulates w1[t1] w2[t2] v in a register while the cell stays the same and adds it
//    into its wave's own LDS copy of the patch when the (wave-uniform) cell changes, so no two lanes ever
//    update the same address.  The wave copies are summed in a fixed order.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "op.hpp"
#include "plan.hpp"
#include "tables.hpp"

namespace {

constexpr int GRID_CHUNK = 4096;   // default visibilities per work item

// The J = 8 gridder: waves per work-group (two streams each).  Two keep a work-group's LDS near 18 KB, so
// that the registers (five waves per SIMD), not LDS, bound the occupancy.
constexpr int grid_mfma_waves(int) { return 2; }

// All J tap weights at s = 2f - 1.  Tap J-1-t at f is tap t at 1 - f (the window is even), and the tap
// polynomials are tabulated with that symmetry, so the pair shares its even and odd parts in s:
// w_t = E(s^2) + s O(s^2), w_(J-1-t) = E(s^2) - s O(s^2) (KB_DEG odd; 2 (KB_DEG - 1) + 2 FMA per pair).
template <int J>
__device__ __forceinline__ void kb_weights(const KBCoef& kc, float s, float* w) {
  static_assert(KB_DEG % 2 == 1, "odd polynomial degree");
  const float u = s * s;
#pragma unroll
  for (int t = 0; t < J / 2; ++t) {
    const float* c = kc.c[t];
    float e = c[KB_DEG - 1], o = c[KB_DEG];
#pragma unroll
    for (int i = KB_DEG - 3; i >= 0; i -= 2) {
      e = fmaf(e, u, c[i]);
      o = fmaf(o, u, c[i + 1]);
    }
    w[t] = fmaf(s, o, e);
    w[J - 1 - t] = fmaf(-s, o, e);
  }
}

// Orders this lane's LDS accesses around a point where lanes of one wave hand data to each other
// through LDS: the compiler reasons per lane and could otherwise move a read of one address above a
// write that another lane makes to it.  One wave's LDS operations execute in program order, so a
// wavefront-scope fence (a compiler barrier that needs no wait instruction) is enough.
__device__ __forceinline__ void wave_lds_order() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Degridding of one item: the tile's padded (T+J-1)^2 grid patch is staged in LDS, then
// V = sum_{t1,t2} w1[t1] w2[t2] X[r0 + t1, c0 + t2] per visibility.
template <int J, int T>
__global__ __launch_bounds__(256) void degrid_kernel(const uint2* __restrict__ coord, const float2* __restrict__ grid,
                                                     float2* __restrict__ out, const uint32_t* __restrict__ oidx,
                                                     const int4* __restrict__ items,
                                                     const int32_t* __restrict__ item_block, int log2K, int log2T,
                                                     const float* __restrict__ scales, KBCoef kc,
                                                     const int32_t* __restrict__ bmask) {
  constexpr int P = T + J - 1;
  constexpr int LO = J / 2 - 1;
  __shared__ float2 patch[P * P];
  const int tid = threadIdx.x;
  const int itx = xcd_block_runs(blockIdx.x, gridDim.x, 16);
  if (bmask && !bmask[item_block[itx]]) return;   // block not selected this iteration: its outputs are kept
  const int4 it = items[itx];
  const int nT = 1 << (log2K - log2T);
  const int kmask = (1 << log2K) - 1;
  const int prob = it.x >> (2 * (log2K - log2T)), tloc = it.x & ((1 << (2 * (log2K - log2T))) - 1);
  const int a0 = (tloc / nT) * T, b0 = (tloc % nT) * T;
  grid += (size_t)prob << (2 * log2K);
  const float scale = scales ? scales[item_block[itx]] : 1.f;
  for (int e = tid; e < P * P; e += 256) {
    const int p1 = e / P, p2 = e - p1 * P;
    patch[e] = grid[(size_t)((a0 - LO + p1) & kmask) * (kmask + 1) + ((b0 - LO + p2) & kmask)];
  }
  __syncthreads();
  const int F = 32 - log2K;
  const uint32_t fmask = (F == 32) ? 0xffffffffu : ((1u << F) - 1u);
  const float fs = ldexpf(1.0f, 1 - F);
  // the item's visibilities interleaved over the threads, so that the coordinate loads and visibility stores
  // coalesce
  for (int j = it.y + tid; j < it.y + it.z; j += 256) {
    const uint2 c = coord[j];
    const int lr = int(c.x >> F) - a0, lc = int(c.y >> F) - b0;
    const float s1 = float(c.x & fmask) * fs - 1.0f;
    const float s2 = float(c.y & fmask) * fs - 1.0f;
    float w1[J], w2[J];
    kb_weights<J>(kc, s1, w1);
    kb_weights<J>(kc, s2, w2);
    float ar = 0.f, ai = 0.f;
    // the window fully unrolled (the row weights w1[t1] stay in registers with static indices; a loop over
    // the rows would select them with compare-and-select chains), two rows per scheduling region: left free,
    // the scheduler hoists all J^2 loads (155 VGPRs, three waves per SIMD at J = 8)
#pragma unroll
    for (int t1 = 0; t1 < J; ++t1) {
      const float2* row = patch + (lr + t1) * P + lc;
      float rr = 0.f, ri = 0.f;
#pragma unroll
      for (int t2 = 0; t2 < J; ++t2) {
        const float2 g = row[t2];
        rr = fmaf(w2[t2], g.x, rr);
        ri = fmaf(w2[t2], g.y, ri);
      }
      ar = fmaf(w1[t1], rr, ar);
      ai = fmaf(w1[t1], ri, ai);
      if (t1 & 1) __asm__ volatile("" : "+v"(ar), "+v"(ai) :: "memory");   // these rows done before the next loads
    }
    out[oidx ? oidx[j] : j] = make_float2(ar * scale, ai * scale);
  }
}

// Gridding of one work item into a private padded patch, written to patches[item slot].
// Wave w owns the w-th quarter of the item and its own copy of the patch.  It walks its
// visibilities in batches of NB = 32.  Phase A (lane l for visibility l mod 32; lanes 0-31 the first
// axis, 32-63 the second) writes a1[t1] = w1[t1] * scale * v and w2[t2] to the wave's LDS rows and marks,
// in a ballot, where the cell changes; 32-entry rows keep the kernel's LDS at 30 KiB (five work-groups per
// CU at J = 8, T = 16).  Phase B
// (one lane per tap (t1, t2)) accumulates w2[t2] * a1[t1] in registers while the cell stays the same;
// at a cell change the finished run is added into the wave's patch copy with a read-modify-write
// (64 lanes, 64 distinct addresses, no other wave on this copy) whose write is deferred to the next
// change so that the read has landed by then.  The wave's cells are non-decreasing, so no later
// read needs a deferred value.  (LDS float atomics would avoid the read but measure several times
// slower here.)  Every sum has a fixed order, so the result is reproducible.  Latency: the next batch's
// coordinates and visibilities are loaded while the current batch is accumulated, and, where the extra
// registers cost no occupancy (J <= 8 with a patch large enough that LDS already caps the occupancy at
// five waves per SIMD, as at J = 8, T = 16), phase B reads the LDS rows of a full batch's next step
// before the products of the current one.
template <int J, int T>
__global__ __launch_bounds__(256) void grid_kernel(const uint2* __restrict__ coord, const float2* __restrict__ vis,
                                                   const uint32_t* __restrict__ vidx, const int4* __restrict__ items,
                                                   const int32_t* __restrict__ item_block, float2* __restrict__ patches,
                                                   int log2K, int log2T, const float* __restrict__ scales, KBCoef kc,
                                                   const int32_t* __restrict__ bmask) {
  constexpr int P = T + J - 1;
  constexpr int PP = P * P;
  constexpr int NQ = (J * J + 63) / 64;   // taps per lane
  __shared__ float2 pat[4][PP];           // one patch copy per wave
  // per wave, tap-major; row pitches of 34 complex / 36 real entries keep every row 16-byte aligned
  // for the 128-bit reads of phase B (two visibilities of aw, four of bw per read) while the rows of
  // different taps land in disjoint LDS banks (row strides of 68 and 36 words); phase A (consecutive
  // lanes) is conflict-free too
  constexpr int NB = 32, AWP = NB + 2, BWP = NB + 4;
  __shared__ __attribute__((aligned(16))) float2 aw[4][J][AWP];  // w1[t1] * scale * v, current NB visibilities
  __shared__ __attribute__((aligned(16))) float bw[4][J + 1][BWP];  // w2[t2]; row J stays 0
  // Phase B reads one step ahead (a second register set: about 30 more VGPRs, five waves per SIMD) only
  // where LDS already limits the occupancy to five work-groups per CU or fewer and a lane has one tap
  constexpr int LDS_BYTES = int(sizeof(pat) + sizeof(aw) + sizeof(bw));
  constexpr bool PIPELINE = NQ == 1 && 160 * 1024 / LDS_BYTES <= 5;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  for (int e = tid; e < 4 * PP; e += 256) (&pat[0][0])[e] = make_float2(0.f, 0.f);
  __syncthreads();
  const int itx = xcd_block_runs(blockIdx.x, gridDim.x, 16);
  int4 it = items[itx];
  if (bmask && !bmask[item_block[itx]]) it.z = 0;   // block not selected: a zero patch, no visibility read
  const int nT = 1 << (log2K - log2T);
  const int prob = it.x >> (2 * (log2K - log2T)), tloc = it.x & ((1 << (2 * (log2K - log2T))) - 1);
  const int a0 = (tloc / nT) * T, b0 = (tloc % nT) * T;
  const float scale = scales ? scales[item_block[itx]] : 1.f;
  const int F = 32 - log2K;
  const uint32_t fmask = (F == 32) ? 0xffffffffu : ((1u << F) - 1u);
  const float fs = ldexpf(1.0f, 1 - F);
  int toff[NQ], tr[NQ], tc[NQ];            // this lane's taps: patch offset from tap (0, 0), row, column
  bool tval[NQ];
  float2 acc[NQ], pend_val[NQ], pend_old[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int t = q * 64 + lane;
    tval[q] = t < J * J;
    tr[q] = tval[q] ? t / J : 0;              // lanes past the last tap read tap (0, 0) with weight 0
    tc[q] = tval[q] ? t % J : J;              // row J of bw is always 0
    toff[q] = tval[q] ? (t / J) * P + t % J : 0;
    acc[q] = pend_val[q] = pend_old[q] = make_float2(0.f, 0.f);
  }
  float2* mypat = pat[wave];
  if (lane < BWP) bw[wave][J][lane] = 0.f;
  int cur = -1, pend = -1;                  // patch offset of tap (0, 0): current run, deferred run
  const int w_lo = it.y + int((int64_t)it.z * wave / 4);
  const int w_hi = it.y + int((int64_t)it.z * (wave + 1) / 4);
  static_assert(NB == 32, "phase B's full-batch schedule covers 32 visibilities");
  const int vl = lane & (NB - 1);           // this lane's visibility in the batch
  const bool ax2 = lane >= NB;              // lanes NB..63 weigh the second axis
  // this lane's coordinate and visibility of the next batch, loaded while the current one is accumulated
  uint2 cn = make_uint2(0u, 0u);
  float2 vn = make_float2(0.f, 0.f);
  auto fetch = [&](int j) {
    if (j < w_hi) {                         // the visibility first: its index may need a load of its own
      if (!ax2) vn = vis[vidx ? vidx[j] : j];
      cn = coord[j];
    }
  };
  fetch(w_lo + vl);
  for (int base = w_lo; base < w_hi; base += NB) {
    const int nb = min(NB, w_hi - base);
    int cell = -1;
    if (vl >= nb) {                         // padding entries contribute exactly zero
      if (!ax2) {
#pragma unroll
        for (int t = 0; t < J; ++t) aw[wave][t][vl] = make_float2(0.f, 0.f);
      } else {
#pragma unroll
        for (int t = 0; t < J; ++t) bw[wave][t][vl] = 0.f;
      }
    } else {                                // phase A
      const uint2 c = cn;
      const float sv = float((ax2 ? c.y : c.x) & fmask) * fs - 1.0f;
      float w[J];
      kb_weights<J>(kc, sv, w);
      if (!ax2) {
        const float2 v = vn;
        const float vr = v.x * scale, vi = v.y * scale;
#pragma unroll
        for (int t = 0; t < J; ++t) aw[wave][t][vl] = make_float2(w[t] * vr, w[t] * vi);
      } else {
#pragma unroll
        for (int t = 0; t < J; ++t) bw[wave][t][vl] = w[t];
      }
      cell = (int(c.x >> F) - a0) * P + (int(c.y >> F) - b0);
    }
    fetch(base + NB + vl);
    // run starts of this batch: lane i starts a run if its cell differs from lane i-1's
    // (lane 0 compares with the run carried over from the previous batch)
    const int prev = __shfl_up(cell, 1);
    const uint64_t starts = __ballot(lane < nb && cell != (lane == 0 ? cur : prev));
    wave_lds_order();                       // phase A rows visible to every lane
    const int nb8 = (nb + 7) & ~7;          // entries up to nb8 exist (padding is zero)
    // phase B, eight visibilities per step; with PIPELINE, in a full batch the LDS reads of the next step
    // are issued before the products of the current one (two register sets)
    float2 av[2][NQ][8];
    float bv[2][NQ][8];
    auto stage = [&](int s, int k) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          const float4 a2 = *(const float4*)&aw[wave][tr[q]][k + u];
          av[s][q][u] = make_float2(a2.x, a2.y);
          av[s][q][u + 1] = make_float2(a2.z, a2.w);
        }
#pragma unroll
        for (int u = 0; u < 8; u += 4) {
          const float4 b4 = *(const float4*)&bw[wave][tc[q]][k + u];
          bv[s][q][u] = b4.x;
          bv[s][q][u + 1] = b4.y;
          bv[s][q][u + 2] = b4.z;
          bv[s][q][u + 3] = b4.w;
        }
      }
    };
    auto step = [&](int s, int k) {
      const uint32_t group = uint32_t(starts >> k) & 0xffu;
      if (group == 0) {                     // no run starts here: straight-line accumulation
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            acc[q].x = fmaf(bv[s][q][u], av[s][q][u].x, acc[q].x);
            acc[q].y = fmaf(bv[s][q][u], av[s][q][u].y, acc[q].y);
          }
        return;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if ((group >> u) & 1) {
          if (pend >= 0) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
              if (tval[q])                  // lanes without a tap must not touch the patch
                mypat[pend + toff[q]] = make_float2(pend_old[q].x + pend_val[q].x, pend_old[q].y + pend_val[q].y);
            wave_lds_order();               // another lane's next read may hit an address just written
          }
          pend = cur;
          if (cur >= 0) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              if (tval[q]) pend_old[q] = mypat[cur + toff[q]];
              pend_val[q] = acc[q];
              acc[q] = make_float2(0.f, 0.f);
            }
          }
          cur = __builtin_amdgcn_readlane(cell, k + u);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          acc[q].x = fmaf(bv[s][q][u], av[s][q][u].x, acc[q].x);
          acc[q].y = fmaf(bv[s][q][u], av[s][q][u].y, acc[q].y);
        }
      }
    };
    if (PIPELINE && nb == NB) {             // a full batch: the schedule is static
      stage(0, 0);
      stage(1, 8);
      step(0, 0);
      stage(0, 16);
      step(1, 8);
      stage(1, 24);
      step(0, 16);
      step(1, 24);
    } else {                                // the wave's last, partial batch
      for (int k = 0; k < nb8; k += 8) {
        stage(0, k);
        step(0, k);
      }
    }
    wave_lds_order();                       // rows of this batch consumed before the next phase A
  }
  if (pend >= 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (tval[q]) mypat[pend + toff[q]] = make_float2(pend_old[q].x + pend_val[q].x, pend_old[q].y + pend_val[q].y);
    wave_lds_order();
  }
  if (cur >= 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (tval[q]) {
        const float2 o = mypat[cur + toff[q]];
        mypat[cur + toff[q]] = make_float2(o.x + acc[q].x, o.y + acc[q].y);
      }
  }
  __syncthreads();
  float2* dst = patches + (size_t)it.w * PP;
  for (int e = tid; e < PP; e += 256) {
    const float2 p0 = pat[0][e], p1 = pat[1][e], p2 = pat[2][e], p3 = pat[3][e];
    dst[e] = make_float2(((p0.x + p1.x) + p2.x) + p3.x, ((p0.y + p1.y) + p2.y) + p3.y);
  }
}

// Gridding with J = 8 on the matrix cores.  v_mfma_f32_4x4x1_16b_f32 forms sixteen independent 4 x 4
// outer products a b^T and adds them to its accumulator: block k takes a[i] from lane 4k + i and b[j] from
// lane 4k + j, and leaves entry (i, j) in accumulator register i of lane 4k + j.  One visibility's 8 x 8 taps,
// real and imaginary part, are eight such blocks: block (r, tb, ub) holds taps t1 = 4 tb + i, t2 = 4 ub + j
// of part r, with a = w1[t1] Re/Im(v) and b = w2[t2].  One instruction therefore grids two visibilities, one
// per half-wave, and each half-wave is an independent stream over its share of the item.
//
// Phase A: each lane computes both axes' weights of one visibility of its stream and stages a (real and
// imaginary rows) and b in LDS, tap-major, so that phase B reads four consecutive visibilities' operands
// with one 128-bit load.  Phase B: while a stream stays in one cell its blocks accumulate in the matrix
// registers; when the cell changes, each of the stream's lanes writes its four sums, added to the values it
// read from the stream's own copy of the patch when the run started, back to the copy, reads the values under
// the next run and restarts from zero (LDS float atomics would serialise over the lanes).  No other lane
// touches those addresses and one wave's LDS operations execute in order, so every entry of a copy is a sum
// in a fixed order; the copies are summed in a fixed order at the end, and the adjoint stays bitwise
// reproducible.
template <int T, int NWV>
__global__ __launch_bounds__(64 * NWV) void grid_mfma_kernel(const uint2* __restrict__ coord,
                                                             const float2* __restrict__ vis,
                                                             const uint32_t* __restrict__ vidx,
                                                             const int4* __restrict__ items,
                                                             const int32_t* __restrict__ item_block,
                                                             const int4* __restrict__ item_rows,
                                                             float2* __restrict__ patches, int log2K, int log2T,
                                                             const float* __restrict__ scales, KBCoef kc,
                                                             const int32_t* __restrict__ bmask) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int J = 8, P = T + J - 1, PP = P * P;
  constexpr int NS = 2 * NWV;             // streams per work-group
  // Each stream's copy of the patch covers only the cell rows its visibilities occupy plus J - 1 (its stream
  // is a contiguous run of the item, sorted by row, so the rows of all streams add up to at most
  // T + NS - 1; an empty stream still gets one row): rows of pitch PR in a pool of RMAX rows, a real and
  // an imaginary plane PL words apart.  PR = 2 (mod 8) and PL = 16 (mod 32) put the 32 addresses one
  // write-back instruction of a stream touches (offsets i + 4 ub + 4 tb PR + r PL) in 32 different banks.
  constexpr int PR = ((P + 5) / 8) * 8 + 2;
  constexpr int RMAX = T + NS - 1 + NS * (J - 1);
  constexpr int PL = ((RMAX * PR + 15) / 32) * 32 + 16;
  constexpr int NB = 16;                  // visibilities per stream and batch (two lanes each in phase A)
  constexpr int SP = NB + 4;              // staging row pitch: rows 4 words apart, 16-byte aligned
  static_assert(PR >= P && PL >= RMAX * PR && NS <= 8, "copy layout");
  __shared__ __attribute__((aligned(16))) float cp[2 * PL];
  // staged per stream and batch: rows a real, a imaginary, b (J each)
  __shared__ __attribute__((aligned(16))) float stg[NWV][2][3 * J][SP];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int h = lane >> 5, ax = (lane >> 4) & 1, jl = lane & 15;   // phase A: visibility jl, axis ax
  const int itx = xcd_block_runs(blockIdx.x, gridDim.x, 16);
  int4 it = items[itx];
  const int4 ir = item_rows[itx];
  if (bmask && !bmask[item_block[itx]]) it.z = 0;   // block not selected: a zero patch, no visibility read
  // the streams' first rows and pool rows (uniform): stream k's rows start at row base[k] of the pool
  int first[NS], base[NS + 1];
  base[0] = 0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    first[k] = ((k < 4 ? ir.x : ir.y) >> (8 * (k & 3))) & 255;
    base[k + 1] = base[k] + (((k < 4 ? ir.z : ir.w) >> (8 * (k & 3))) & 255) + J - 1;
  }
  const int s = wave * 2 + h;             // this lane's stream
  const int lo = it.y + int((int64_t)it.z * s / NS), hi = it.y + int((int64_t)it.z * (s + 1) / NS);
  const int nbatch = (it.z + NS * NB - 1) / (NS * NB);   // batches of the longest stream
  // Loads are unconditional (past the stream's end they read the item's first entry, which always exists,
  // and the value is discarded where it is used), so that nothing waits for them before they are used.
  uint2 cn;
  float2 vn;
  auto fetch = [&](int b) {
    const int j = lo + b * NB + jl;
    const int jj = j < hi ? j : it.y;
    vn = vis[vidx ? vidx[jj] : jj];
    cn = coord[jj];
  };
  fetch(0);                                 // in flight while the pool is cleared
  {
    const int n4 = (base[NS] * PR + 3) / 4;   // every stream's rows
    float4* c0 = reinterpret_cast<float4*>(cp);
    float4* c1 = reinterpret_cast<float4*>(cp + PL);
    for (int e = tid; e < n4; e += 64 * NWV) {
      c0[e] = make_float4(0.f, 0.f, 0.f, 0.f);
      c1[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  __syncthreads();
  const int nT = 1 << (log2K - log2T);
  const int tloc = it.x & ((1 << (2 * (log2K - log2T))) - 1);
  const int a0 = (tloc / nT) * T, b0 = (tloc % nT) * T;
  const float scale = scales ? scales[item_block[itx]] : 1.f;
  const int F = 32 - log2K;
  const uint32_t fmask = (F == 32) ? 0xffffffffu : ((1u << F) - 1u);
  const float fs = ldexpf(1.0f, 1 - F);
  int myfirst = 0, mybase = 0;             // this lane's stream (static indices: no indexed registers)
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    if (k == s) myfirst = first[k];
    if (k < s) mybase = base[k + 1];
  }
  // phase B roles: block (r, tb, ub) of this half, row/column i4
  const int bl = (lane >> 2) & 7, r = bl >> 2, tb = (bl >> 1) & 1, ub = bl & 1, i4 = lane & 3;
  const float* arow = &stg[wave][h][r * J + tb * 4 + i4][0];
  const float* brow = &stg[wave][h][2 * J + ub * 4 + i4][0];
  float* const mycp = cp + r * PL + (mybase + tb * 4) * PR + ub * 4 + i4;
  float* wcol = &stg[wave][h][0][jl];     // phase A: this lane's column
  // The current run of this lane's stream: this lane's first copy address under it and the copy's values
  // under it plus the run's products so far (matrix accumulators, loaded from the copy when the run started).
  // A stream starts at cell offset 0 with zeros, which is what the cleared copy holds there, so its first
  // write-back needs no special case.
  float* cur = mycp;
  int curv = 0;                             // cell offset of the current run (first-axis lanes of phase A)
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int b = 0; b < nbatch; ++b) {
    const bool valid = lo + b * NB + jl < hi;
    // past the stream's end: weight 0 (coordinate 0 keeps the weights finite)
    const uint2 c = valid ? cn : make_uint2(0u, 0u);
    const float2 v = valid ? vn : make_float2(0.f, 0.f);
    fetch(b + 1);                           // the next batch's loads stay in flight through this one
    // this lane's axis: J weights; the first axis's lanes scale them by the visibility (a, real and imaginary
    // rows), the second axis's lanes store them as they are (b)
    float w[J];
    kb_weights<J>(kc, float((ax ? c.y : c.x) & fmask) * fs - 1.0f, w);
    const int cell = valid ? (int(c.x >> F) - a0 - myfirst) * PR + (int(c.y >> F) - b0) : -1;
    if (!ax) {
      const float vr = v.x * scale, vi = v.y * scale;
#pragma unroll
      for (int t = 0; t < J; ++t) {
        wcol[t * SP] = w[t] * vr;
        wcol[(J + t) * SP] = w[t] * vi;
      }
    } else {
#pragma unroll
      for (int t = 0; t < J; ++t) wcol[(2 * J + t) * SP] = w[t];
    }
    // the previous visibility's cell: lane - 1 within each row of 16 lanes (DPP row_shr:1; lane 0 of a row
    // keeps its own value and takes curv instead)
    const int left = __builtin_amdgcn_update_dpp(cell, cell, 0x111, 0xf, 0xf, false);
    const int prev = jl == 0 ? curv : left;
    // bit 32 h + j: stream h starts a run at its visibility j (the first axis's lanes decide)
    const uint64_t starts = __ballot(!ax && valid && cell != prev);
    const uint32_t any = uint32_t(starts) | uint32_t(starts >> 32);
    // the cell of the stream's last visibility of this batch, for the next batch's first comparison (when
    // that visibility is past the stream's end, so are all later ones, and the value is never used)
    {
      const int c0 = __builtin_amdgcn_readlane(cell, NB - 1), c1 = __builtin_amdgcn_readlane(cell, 32 + NB - 1);
      curv = h ? c1 : c0;
    }
    wave_lds_order();                       // staged rows visible to every lane
    // every operand of the batch in registers (128-bit reads), so that the steps never wait for LDS except for
    // the values under a new run
    float av[NB], bv[NB];
#pragma unroll
    for (int g = 0; g < NB / 4; ++g) {
      const float4 a4 = *(const float4*)(arow + 4 * g), b4 = *(const float4*)(brow + 4 * g);
      av[4 * g] = a4.x, av[4 * g + 1] = a4.y, av[4 * g + 2] = a4.z, av[4 * g + 3] = a4.w;
      bv[4 * g] = b4.x, bv[4 * g + 1] = b4.y, bv[4 * g + 2] = b4.z, bv[4 * g + 3] = b4.w;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      // (most steps continue a run: the write-back is laid out away from the straight-line path, so that
      // those steps do not branch)
      if (__builtin_expect((any >> j) & 1, 0)) {   // a stream of this wave starts a run here
        const uint64_t sel = (((starts >> j) & 1) ? 0x00000000ffffffffull : 0ull) |
                             (((starts >> (32 + j)) & 1) ? 0xffffffff00000000ull : 0ull);
        // the new run's cell offsets of both streams (uniform values, read outside the lane mask)
        const int n0 = __builtin_amdgcn_readlane(cell, j), n1 = __builtin_amdgcn_readlane(cell, 32 + j);
        if (__builtin_amdgcn_inverse_ballot_w64(sel)) {   // the lanes of the streams that start a run
          // write the finished run back (the copy's values plus its products), then load the values under
          // the new run into the accumulators: the run's products add to them in order
#pragma unroll
          for (int q = 0; q < 4; ++q) cur[q * PR] = acc[q];
          wave_lds_order();                 // the new run's window may overlap: read after the write
          cur = mycp + (h ? n1 : n0);
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] = cur[q * PR];
          // wait here for the LDS reads (lgkmcnt 0, the other counters left alone), so that the steps after the
          // join do not each wait for every read of the batch
          __builtin_amdgcn_s_waitcnt(0xC07F);
        }
      }
      acc = __builtin_amdgcn_mfma_f32_4x4x1f32(av[j], bv[j], acc, 0, 0, 0);
    }
    wave_lds_order();                       // staged rows consumed before the next phase A
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) cur[q * PR] = acc[q];
  __syncthreads();
  float2* dst = patches + (size_t)it.w * PP;
  for (int e = tid; e < PP; e += 64 * NWV) {
    const int pr = e / P, pc = e - pr * P;
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int k = 0; k < NS; ++k) {        // the streams whose rows cover this one, in stream order
      const int d = pr - first[k];
      if (d >= 0 && d < base[k + 1] - base[k]) {
        const int o = (base[k] + d) * PR + pc;
        re += cp[o];
        im += cp[PL + o];
      }
    }
    dst[e] = make_float2(re, im);
  }
}

// The sum of one cell over the item patches of the neighbour tiles with row offsets DA0..DA1 (n = 3 (da + 1) +
// (db + 1), in order of n; each tile's items in slot order).  The first item's value of every neighbour is
// loaded before any is summed, so those loads are in flight together; the load is issued for every neighbour
// (slot 0 of the patch array, which always exists, where the neighbour has no item covering the cell) and its
// value is replaced by +0, which leaves the sum unchanged since the sum is never -0.
template <int J, int T, int DA0, int DA1>
__device__ __forceinline__ float2 fold_cell(const float2* __restrict__ patches, const int* __restrict__ tile_items,
                                            int nT, int a, int b, int l1, int l2) {
  constexpr int P = T + J - 1;
  constexpr int LO = J / 2 - 1;
  constexpr int NN = 3 * (DA1 - DA0 + 1);
  int src[NN], n0[NN], n1[NN];
  float2 first[NN];
#pragma unroll
  for (int k = 0; k < NN; ++k) {   // the neighbours' slot ranges (uniform: scalar loads, issued together)
    const int da = DA0 + k / 3, db = k % 3 - 1;
    const int t2 = ((a + da) & (nT - 1)) * nT + ((b + db) & (nT - 1));   // nT is a power of two
    n0[k] = tile_items[t2];
    n1[k] = tile_items[t2 + 1];
  }
#pragma unroll
  for (int k = 0; k < NN; ++k) {
    const int da = DA0 + k / 3, db = k % 3 - 1;
    const int p1 = l1 - da * T + LO, p2 = l2 - db * T + LO;
    const bool cover = p1 >= 0 && p1 < P && p2 >= 0 && p2 < P;
    src[k] = p1 * P + p2;
    if (!cover) n1[k] = n0[k];                      // no items where the patch does not cover the cell
    const bool has = n0[k] < n1[k];
    const float2 v = patches[has ? (size_t)n0[k] * (P * P) + src[k] : 0];
    // the mask goes through an empty asm so that the compiler does not turn the load back into a
    // conditional one (which would then be waited for before the next neighbour's load)
    int m = has ? -1 : 0;
    asm volatile("" : "+v"(m));
    first[k] = make_float2(__int_as_float(__float_as_int(v.x) & m), __int_as_float(__float_as_int(v.y) & m));
  }
  float sr = 0.f, si = 0.f;
#pragma unroll
  for (int k = 0; k < NN; ++k) {
    sr += first[k].x;
    si += first[k].y;
    const float2* p = patches + src[k];
    int i = n0[k] + 1;
    for (; i + 4 <= n1[k]; i += 4) {   // four loads in flight
      const float2 v0 = p[(size_t)i * (P * P)], v1 = p[(size_t)(i + 1) * (P * P)];
      const float2 v2 = p[(size_t)(i + 2) * (P * P)], v3 = p[(size_t)(i + 3) * (P * P)];
      sr += v0.x;
      si += v0.y;
      sr += v1.x;
      si += v1.y;
      sr += v2.x;
      si += v2.y;
      sr += v3.x;
      si += v3.y;
    }
    for (; i < n1[k]; ++i) {
      const float2 v = p[(size_t)i * (P * P)];
      sr += v.x;
      si += v.y;
    }
  }
  return make_float2(sr, si);
}

// Each grid cell = sum over the tiles whose padded patch covers it (3 x 3 neighbourhood, fixed order)
// of that tile's item patches (slot order).  One work-group per group of 256 cells of a tile.  A patch reaches
// J/2 rows into the tile below its own and J/2 - 1 into the one above, so a wave whose cell rows lie clear of
// both tile edges reads only the neighbours of its own tile row (da = 0); the neighbours it skips would add
// +0 (no item of theirs covers its cells), so every cell keeps the same sum.
template <int J, int T>
__global__ __launch_bounds__(256) void fold_kernel(const float2* __restrict__ patches, const int* __restrict__ tile_items,
                                                   float2* __restrict__ grid, int log2K, int log2T) {
  constexpr int G = (T * T + 255) / 256;   // work-groups per tile
  const int nT = 1 << (log2K - log2T);
  const int K = 1 << log2K;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int gtile = blk / G;                 // problem * nT^2 + tile
  const int e = (blk % G) * 256 + threadIdx.x;
  if (e >= T * T) return;
  const int prob = gtile / (nT * nT), tile = gtile - prob * nT * nT;
  const int a = tile / nT, b = tile % nT;
  tile_items += prob * nT * nT;
  grid += (size_t)prob * K * K;
  const int l1 = e / T, l2 = e % T;
  // the wave's first and last cell rows (wave-uniform)
  const int e0 = e & ~63;
  const int r0 = e0 / T, r1 = min(e0 + 63, T * T - 1) / T;
  const bool up = r0 < J / 2;                 // rows reached by the patch of the tile above (da = -1)
  const bool down = r1 >= T - J / 2 + 1;      // rows reached by the patch of the tile below (da = +1)
  float2 v;
  if (up && down) v = fold_cell<J, T, -1, 1>(patches, tile_items, nT, a, b, l1, l2);
  else if (up) v = fold_cell<J, T, -1, 0>(patches, tile_items, nT, a, b, l1, l2);
  else if (down) v = fold_cell<J, T, 0, 1>(patches, tile_items, nT, a, b, l1, l2);
  else v = fold_cell<J, T, 0, 0>(patches, tile_items, nT, a, b, l1, l2);
  grid[(size_t)(a * T + l1) * K + (b * T + l2)] = v;
}

__global__ void gather_kernel(const float2* __restrict__ src, const uint32_t* __restrict__ idx, float2* __restrict__ dst,
                              int64_t M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) dst[i] = src[idx[i]];
}

__global__ void scatter_kernel(const float2* __restrict__ src, const uint32_t* __restrict__ idx, float2* __restrict__ dst,
                               int64_t M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) dst[idx[i]] = src[i];
}

template <int J, int T>
sh_status launch_degrid_T(sh_op op, const float2* grid, float2* out, const uint32_t* oidx, const float* scales,
                          const int32_t* bmask, hipStream_t st) {
  hipLaunchKernelGGL((degrid_kernel<J, T>), dim3((unsigned)op->n_items), dim3(256), 0, st, op->coord.ptr, grid, out,
                     oidx, op->items.ptr, op->item_block.ptr, op->log2K, op->log2T, scales, op->kb, bmask);
  SH_LAUNCHED();
  return SH_OK;
}

template <int J>
sh_status launch_degrid(sh_op op, const float2* grid, float2* out, const uint32_t* oidx, const float* scales,
                        const int32_t* bmask, hipStream_t st) {
  switch (op->T) {
    case 8: return launch_degrid_T<J, 8>(op, grid, out, oidx, scales, bmask, st);
    case 16: return launch_degrid_T<J, 16>(op, grid, out, oidx, scales, bmask, st);
    case 32: return launch_degrid_T<J, 32>(op, grid, out, oidx, scales, bmask, st);
  }
  sh::set_error("unsupported tile %d", op->T);
  return SH_EUNSUPPORTED;
}

template <int J, int T>
sh_status launch_grid_T(sh_op op, const float2* vis, const uint32_t* vidx, const float* scales, const int32_t* bmask,
                        hipStream_t st) {
  {
    sh::ProfScope ps("grid", st);
    if constexpr (J == 8) {
      constexpr int NWV = grid_mfma_waves(T);
      hipLaunchKernelGGL((grid_mfma_kernel<T, NWV>), dim3((unsigned)op->n_items), dim3(64 * NWV), 0, st,
                         op->coord.ptr, vis, vidx, op->items.ptr, op->item_block.ptr, op->item_rows.ptr,
                         op->patches.ptr, op->log2K, op->log2T, scales, op->kb, bmask);
    } else {
      hipLaunchKernelGGL((grid_kernel<J, T>), dim3((unsigned)op->n_items), dim3(256), 0, st, op->coord.ptr, vis,
                         vidx, op->items.ptr, op->item_block.ptr, op->patches.ptr, op->log2K, op->log2T, scales,
                         op->kb, bmask);
    }
    SH_LAUNCHED();
  }
  sh::ProfScope ps("fold", st);
  constexpr int G = (T * T + 255) / 256;
  hipLaunchKernelGGL((fold_kernel<J, T>), dim3((unsigned)(op->P * op->nT * op->nT * G)), dim3(256), 0, st, op->patches.ptr,
                     op->tile_items.ptr, op->grid.ptr, op->log2K, op->log2T);
  SH_LAUNCHED();
  return SH_OK;
}

template <int J>
sh_status launch_grid(sh_op op, const float2* vis, const uint32_t* vidx, const float* scales, const int32_t* bmask,
                      hipStream_t st) {
  switch (op->T) {
    case 8: return launch_grid_T<J, 8>(op, vis, vidx, scales, bmask, st);
    case 16: return launch_grid_T<J, 16>(op, vis, vidx, scales, bmask, st);
    case 32: return launch_grid_T<J, 32>(op, vis, vidx, scales, bmask, st);
  }
  sh::set_error("unsupported tile %d", op->T);
  return SH_EUNSUPPORTED;
}

}  // namespace

namespace sh {

sh_status phi_forward(sh_op op, const float* x, float2* vis, bool user_order, const float* scales, hipStream_t st,
                      const int32_t* bmask) {
  SH_TRY(fft_forward_2d(op, x, op->grid.ptr, st));
  ProfScope ps("degrid", st);
  const uint32_t* oi = user_order ? op->perm.ptr : nullptr;
  switch (op->J) {
#define SH_J(JJ) \
  case JJ: return launch_degrid<JJ>(op, op->grid.ptr, vis, oi, scales, bmask, st);
    SH_J(2) SH_J(4) SH_J(6) SH_J(8) SH_J(10) SH_J(12) SH_J(14) SH_J(16)
#undef SH_J
  }
  set_error("unsupported J");
  return SH_EUNSUPPORTED;
}

sh_status phi_adjoint(sh_op op, const float2* vis, float* x, bool user_order, const float* scales, hipStream_t st,
                      const int32_t* bmask) {
  const uint32_t* vi = user_order ? op->perm.ptr : nullptr;
  sh_status s = SH_EUNSUPPORTED;
  switch (op->J) {
#define SH_J(JJ) \
  case JJ: s = launch_grid<JJ>(op, vis, vi, scales, bmask, st); break;
    SH_J(2) SH_J(4) SH_J(6) SH_J(8) SH_J(10) SH_J(12) SH_J(14) SH_J(16)
#undef SH_J
  }
  SH_TRY(s);
  return fft_adjoint_2d(op, op->grid.ptr, x, st);
}

}  // namespace sh

// ------------------------------------------------------------------------------------------------
// Planner and C ABI
// ------------------------------------------------------------------------------------------------

static sh_status op_build(sh_op op, const double* uv, const int64_t* offs) {
  const int64_t M = op->M;
  const int K = op->K;
  sh::PlanShape shape{M, K, op->log2K, op->T, op->log2T, op->nT, op->P, op->R, op->chunk,
                      op->J == 8 ? 2 * grid_mfma_waves(op->T) : 0};
  sh::HostPlan h;
  sh::plan_host(shape, uv, offs, op->block_prob.data(), h);
  op->n_items = (int64_t)h.items.size();
  op->n_sparse = op->n_items;   // every item takes the interleaved degridder
  op->max_items_per_tile = h.max_items_per_tile;
  op->chunk_first = h.chunk_first;
  op->n_chunks = (int64_t)h.chunks.size();

  SH_TRY(op->coord.upload(h.coord));
  SH_TRY(op->perm.upload(h.perm));
  SH_TRY(op->items.upload(h.items));
  SH_TRY(op->item_block.upload(h.item_block));
  if (!h.item_rows.empty()) SH_TRY(op->item_rows.upload(h.item_rows));
  SH_TRY(op->tile_items.upload(h.tile_items));
  SH_TRY(op->chunks.upload(h.chunks));
  SH_TRY(op->chunk_first_d.upload(op->chunk_first));
  SH_TRY(op->block_prob_d.upload(op->block_prob));
  SH_TRY(op->partials.alloc(2 * std::max<int64_t>(op->n_chunks, 1)));
  // tables
  std::vector<float> dp(op->n);
  for (int r = 0; r < op->n; ++r) dp[r] = float(1.0 / sh::kb_transform(double(r - op->n / 2) / K, op->J, op->beta));
  SH_TRY(op->deapod.upload(dp));
  std::vector<float2> tw;
  sh::fft_twiddles(K, tw);
  SH_TRY(op->tw.upload(tw));
  // scratch
  const int P = op->T + op->J - 1;
  SH_TRY(op->grid.alloc((size_t)op->P * K * K));
  SH_TRY(op->half.alloc((size_t)op->P * op->n * K));
  SH_TRY(op->patches.alloc((size_t)std::max<int64_t>(op->n_items, 1) * P * P));
  SH_TRY(op->vis_tmp.alloc((size_t)M));
  return SH_OK;
}

extern "C" {

sh_status sh_op_create_batched(const double* uv, const int64_t* M_p, int32_t P, int32_t n, int32_t oversample,
                               int32_t kernel_width, const int64_t* block_offsets, const int32_t* R_p, int32_t tile,
                               int32_t chunk, sh_op* out) {
  SH_REQUIRE(out != nullptr, "out is NULL");
  *out = nullptr;
  SH_REQUIRE(uv != nullptr && block_offsets != nullptr && M_p != nullptr && R_p != nullptr, "NULL argument");
  SH_REQUIRE(P >= 1 && P <= 4096, "P must be in [1, 4096], got %d", P);
  int64_t M = 0;
  int64_t R = 0;
  for (int p = 0; p < P; ++p) {
    SH_REQUIRE(M_p[p] >= 1, "problem %d has no visibilities", p);
    SH_REQUIRE(R_p[p] >= 1 && R_p[p] <= M_p[p], "problem %d: R must be in [1, M]", p);
    M += M_p[p];
    R += R_p[p];
  }
  SH_REQUIRE(M < (int64_t(1) << 31), "total M must be < 2^31, got %lld", (long long)M);
  SH_REQUIRE(sh::is_pow2(n) && n >= 16 && n <= 4096, "n must be a power of two in [16, 4096], got %d", n);
  SH_REQUIRE(oversample == 2 || oversample == 4, "oversample must be 2 or 4, got %d", oversample);
  SH_REQUIRE(kernel_width >= 2 && kernel_width <= 16 && kernel_width % 2 == 0, "J must be even in [2, 16], got %d",
             kernel_width);
  SH_REQUIRE(block_offsets[0] == 0 && block_offsets[R] == M, "block offsets must run from 0 to M");
  for (int64_t i = 0; i < R; ++i)
    SH_REQUIRE(block_offsets[i + 1] > block_offsets[i], "block offsets must be strictly increasing (block %lld)",
               (long long)i);
  {  // every problem's blocks cover exactly its visibility range
    int64_t vb = 0, bi = 0;
    for (int p = 0; p < P; ++p) {
      SH_REQUIRE(block_offsets[bi] == vb && block_offsets[bi + R_p[p]] == vb + M_p[p],
                 "blocks of problem %d must cover its visibilities exactly", p);
      vb += M_p[p];
      bi += R_p[p];
    }
  }
  for (int64_t m = 0; m < 2 * M; ++m)
    SH_REQUIRE(std::isfinite(uv[m]) && uv[m] >= -M_PI && uv[m] < M_PI, "uv[%lld] = %g outside [-pi, pi)",
               (long long)m, uv[m]);
  const int K = n * oversample;
  SH_REQUIRE(K <= 8192, "grid side alpha*n must be <= 8192");
  SH_REQUIRE(tile == 0 || tile == 8 || tile == 16 || tile == 32, "tile must be 0 (auto), 8, 16 or 32");
  SH_REQUIRE(chunk == 0 || (chunk >= 64 && chunk <= (1 << 20)), "chunk must be 0 (auto) or in [64, 2^20]");
  int T = tile ? tile : std::min(16, K / 4);
  while (T < kernel_width / 2) T *= 2;
  SH_REQUIRE(K / T >= 3, "grid side %d needs at least 3 tiles of %d cells", K, T);
  sh_op op = new (std::nothrow) sh_op_s();
  if (!op) {
    sh::set_error("host allocation failed");
    return SH_ENOMEM;
  }
  op->P = P;
  op->M = M;
  op->n = n;
  op->alpha = oversample;
  op->K = K;
  op->log2K = sh::ilog2(K);
  op->J = kernel_width;
  op->R = (int)R;
  op->T = T;
  op->chunk = chunk ? chunk : GRID_CHUNK;
  op->log2T = sh::ilog2(op->T);
  op->nT = K / op->T;
  op->beta = sh::kb_beta(kernel_width, oversample);
  float coef[16 * (KB_DEG + 1)];
  sh::kb_tap_polys(kernel_width, op->beta, KB_DEG, coef);
  for (int t = 0; t < kernel_width; ++t)
    for (int i = 0; i <= KB_DEG; ++i) op->kb.c[t][i] = coef[t * (KB_DEG + 1) + i];
  op->offsets.assign(block_offsets, block_offsets + R + 1);
  op->vis_off.assign(P + 1, 0);
  op->block_off.assign(P + 1, 0);
  op->block_prob.resize(R);
  for (int p = 0; p < P; ++p) {
    op->vis_off[p + 1] = op->vis_off[p] + M_p[p];
    op->block_off[p + 1] = op->block_off[p] + R_p[p];
    for (int b = op->block_off[p]; b < op->block_off[p + 1]; ++b) op->block_prob[b] = p;
  }
  sh_status s = op_build(op, uv, block_offsets);
  if (s != SH_OK) {
    delete op;
    return s;
  }
  *out = op;
  return SH_OK;
}

sh_status sh_op_create_tuned(const double* uv, int64_t M, int32_t n, int32_t oversample, int32_t kernel_width,
                             const int64_t* block_offsets, int32_t R, int32_t tile, int32_t chunk, sh_op* out) {
  SH_REQUIRE(M >= 1 && M < (int64_t(1) << 31), "M must be in [1, 2^31), got %lld", (long long)M);
  SH_REQUIRE(R >= 1 && R <= M, "R must be in [1, M], got %d", R);
  return sh_op_create_batched(uv, &M, 1, n, oversample, kernel_width, block_offsets, &R, tile, chunk, out);
}

sh_status sh_op_create(const double* uv, int64_t M, int32_t n, int32_t oversample, int32_t kernel_width,
                       const int64_t* block_offsets, int32_t R, sh_op* out) {
  return sh_op_create_tuned(uv, M, n, oversample, kernel_width, block_offsets, R, 0, 0, out);
}

sh_status sh_op_create_stream(const double* uv, int64_t M, int32_t n, int32_t oversample, int32_t kernel_width,
                              const int64_t* block_offsets, int32_t R, int32_t tile, int32_t chunk, void* stream,
                              sh_op* out) {
  sh::UploadStreamScope scope((hipStream_t)stream);
  return sh_op_create_tuned(uv, M, n, oversample, kernel_width, block_offsets, R, tile, chunk, out);
}

sh_status sh_op_destroy(sh_op op) {
  delete op;
  return SH_OK;
}

sh_status sh_op_query(sh_op op, int64_t out[10]) {
  SH_REQUIRE(op && out, "NULL argument");
  out[0] = op->M;
  out[1] = op->n;
  out[2] = op->K;
  out[3] = op->J;
  out[4] = op->R;
  out[5] = op->n_items;
  out[6] = op->T;
  out[7] = op->max_items_per_tile;
  out[8] = op->P;
  out[9] = op->n_sparse;
  return SH_OK;
}

sh_status sh_op_block_offsets(sh_op op, int64_t* offsets_out) {
  SH_REQUIRE(op && offsets_out, "NULL argument");
  std::copy(op->offsets.begin(), op->offsets.end(), offsets_out);
  return SH_OK;
}

sh_status sh_op_permutation(sh_op op, int64_t* perm_out) {
  SH_REQUIRE(op && perm_out, "NULL argument");
  std::vector<uint32_t> p(op->M);
  SH_HIP(hipMemcpy(p.data(), op->perm.ptr, op->M * sizeof(uint32_t), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < op->M; ++i) perm_out[i] = p[i];
  return SH_OK;
}

sh_status sh_phi_fwd(sh_op op, const float* x, float* vis, void* stream) {
  SH_REQUIRE(op && x && vis, "NULL argument");
  return sh::phi_forward(op, x, (float2*)vis, true, nullptr, (hipStream_t)stream);
}

sh_status sh_phi_adj(sh_op op, const float* vis, float* x, void* stream) {
  SH_REQUIRE(op && x && vis, "NULL argument");
  return sh::phi_adjoint(op, (const float2*)vis, x, true, nullptr, (hipStream_t)stream);
}

sh_status sh_phi_fwd_internal(sh_op op, const float* x, float* vis, void* stream) {
  SH_REQUIRE(op && x && vis, "NULL argument");
  return sh::phi_forward(op, x, (float2*)vis, false, nullptr, (hipStream_t)stream);
}

sh_status sh_phi_adj_internal(sh_op op, const float* vis, float* x, void* stream) {
  SH_REQUIRE(op && x && vis, "NULL argument");
  return sh::phi_adjoint(op, (const float2*)vis, x, false, nullptr, (hipStream_t)stream);
}

sh_status sh_vis_to_internal(sh_op op, const float* user, float* internal, void* stream) {
  SH_REQUIRE(op && user && internal && user != internal, "NULL or aliased argument");
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)sh::cdiv(op->M, 256)), dim3(256), 0, (hipStream_t)stream,
                     (const float2*)user, op->perm.ptr, (float2*)internal, op->M);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status sh_vis_to_user(sh_op op, const float* internal, float* user, void* stream) {
  SH_REQUIRE(op && user && internal && user != internal, "NULL or aliased argument");
  hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)sh::cdiv(op->M, 256)), dim3(256), 0, (hipStream_t)stream,
                     (const float2*)internal, op->perm.ptr, (float2*)user, op->M);
  SH_LAUNCHED();
  return SH_OK;
}

}  // extern "C"
