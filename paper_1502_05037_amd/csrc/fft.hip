// LDS Stockham FFT passes of the NUFFT measurement operator.
//
// Phi = G F Z S: the n x n image is deapodised (S), placed on the K x K grid at index offset mod K
// (Z) and transformed by the unnormalised 2D DFT F, exp(-2 pi i k.n / K).  Only n of the K grid
// rows and columns are non-zero on input, so the forward transform runs over the n image rows
// (row pass, pruned input) and then over all K columns (column pass, pruned input).  The adjoint
// F^H runs the column pass over all K columns keeping only the n needed rows, then the row pass
// over those n rows keeping the n needed columns, fused with the crop, the deapodisation and Re().
//
// Each work-group transforms B sequences of length L in LDS with self-sorting (Stockham) radix-8
// stages and one radix-4 or radix-2 stage; twiddles come from a float64-derived table.  The same
// passes without deapodisation, and an unpruned forward 2D transform of a dense K x K array, serve
// the Toeplitz form of Phi^dagger Phi.
#include <algorithm>

#include "op.hpp"

namespace {

// COLS_TOEP: column pass of the Toeplitz normal operator (forward DFT of a pruned column, product with
// the transposed kernel spectrum, inverse DFT, keep the n needed rows).  ROWS_ADJ_H: ROWS_ADJ on rows
// of which only columns 0..K/2 were written, the rest following from Hermitian symmetry.
enum Mode {
  ROWS_FWD = 0, COLS_FWD = 1, COLS_ADJ = 2, ROWS_ADJ = 3, FULL_ROWS = 4, FULL_COLS = 5, COLS_TOEP = 6, ROWS_ADJ_H = 7
};

template <bool INV>
__device__ __forceinline__ float2 rot_mi(float2 a) {  // multiply by -i (forward) or +i (inverse)
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (R == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const float2 t2 = cadd(v[1], v[3]), t3 = rot_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  } else {  // R == 8: two radix-4 halves combined with w^q, w = exp(-+ 2 pi i / 8)
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft<4, INV>(e);
    dft<4, INV>(o);
    const float h = 0.70710678118654752f;
    const float2 o1 = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                          : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    const float2 o2 = rot_mi<INV>(o[2]);
    const float2 o3 = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                          : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
}

// LDS slot of element i of a sequence: the low four bits of i are XOR-permuted by bits 4-6 of i and by the
// sequence's tag sx (bits 2-3), a bijection inside every group of 16 elements (L >= 16).  Without it the first
// radix-8 stage, whose threads write eight consecutive elements each, puts every second thread of a 16-lane
// group in the same banks, and the column passes, which load and store their B sequences element by element
// side by side, put the B sequences' elements in the same banks.
__device__ __forceinline__ int swz(int i, int sx) { return i ^ ((i >> 4) & 7) ^ sx; }
template <int L>
__device__ __forceinline__ int slot(int b, int i) { return b * L + swz(i, (b & 3) << 2); }

// One Stockham stage of radix R over a length-L sequence in LDS (all threads of the sequence).
template <int L, int R, bool INV>
__device__ __forceinline__ void stage(float2* buf, const float2* __restrict__ tw, int Ns, int lt, int tpt, int sx) {
  constexpr int NB = L / R;                      // butterflies per sequence
  constexpr int PER = (NB + L / 8 - 1) / (L / 8); // butterflies per thread (tpt = L/8)
  float2 v[PER][R], w[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = lt + q * tpt;
#pragma unroll
    for (int r = 0; r < R; ++r) v[q][r] = buf[swz(j + r * NB, sx)];
  }
  // the twiddles do not depend on the sequence: their loads are issued before the barrier, so that they are in
  // flight with the LDS reads (the first stage, Ns = 1, has none)
  if (Ns > 1) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int k = (lt + q * tpt) % Ns;
      const int step = L / (Ns * R);
#pragma unroll
      for (int r = 1; r < R; ++r) w[q][r] = tw[r * k * step];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = lt + q * tpt;
    const int k = j % Ns;
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 t = w[q][r];
        if (INV) t.y = -t.y;
        v[q][r] = cmul(v[q][r], t);
      }
    }
    dft<R, INV>(v[q]);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[swz(base + r * Ns, sx)] = v[q][r];
  }
  __syncthreads();
}

template <int L, bool INV>
__device__ __forceinline__ void fft_lds(float2* buf, const float2* __restrict__ tw, int lt, int sx) {
  constexpr int TPT = L / 8;
  int Ns = 1;
  constexpr int LOG = __builtin_ctz(L);
  constexpr int N8 = LOG / 3;
  constexpr int REM = LOG % 3;
#pragma unroll
  for (int s = 0; s < N8; ++s) {
    stage<L, 8, INV>(buf, tw, Ns, lt, TPT, sx);
    Ns *= 8;
  }
  if constexpr (REM == 2) stage<L, 4, INV>(buf, tw, Ns, lt, TPT, sx);
  if constexpr (REM == 1) stage<L, 2, INV>(buf, tw, Ns, lt, TPT, sx);
}

// B sequences of length L per work-group, L/8 threads each.
template <int L, int B, int MODE>
__global__ __launch_bounds__(B * L / 8) void fft_pass(const void* __restrict__ in, void* __restrict__ out,
                                                      const float2* __restrict__ tw,
                                                      const float* __restrict__ deapod, int n, int per) {
  extern __shared__ float2 lds[];
  constexpr bool INV = (MODE == COLS_ADJ || MODE == ROWS_ADJ || MODE == ROWS_ADJ_H);
  constexpr int NT = B * L / 8;
  const int tid = threadIdx.x;
  const int K = L;                    // grid side
  // `per` sequences per problem (n rows or K columns); B divides per, so a block stays in one problem
  const int gseq = xcd_block(blockIdx.x, gridDim.x) * B;
  const int prob = gseq / per;
  const int seq0 = gseq - prob * per;  // first row (row modes) or column (column modes) of the problem
  const int half = n / 2;
  const size_t img = (size_t)n * n, hk = (size_t)n * K, gk = (size_t)K * K;
  if constexpr (MODE == ROWS_FWD) {
    in = (const float*)in + prob * img;
    out = (float2*)out + prob * hk;
  } else if constexpr (MODE == COLS_FWD) {
    in = (const float2*)in + prob * hk;
    out = (float2*)out + prob * gk;
  } else if constexpr (MODE == COLS_ADJ) {
    in = (const float2*)in + prob * gk;
    out = (float2*)out + prob * hk;
  } else if constexpr (MODE == FULL_ROWS || MODE == FULL_COLS) {
    in = (const float2*)in + prob * gk;
    out = (float2*)out + prob * gk;
  } else if constexpr (MODE == COLS_TOEP) {
    in = (const float2*)in + prob * hk;
    out = (float2*)out + prob * hk;
    deapod += prob * gk;              // here: the problem's kernel spectrum, transposed (column-major)
  } else {
    in = (const float2*)in + prob * hk;
    out = (float*)out + prob * img;
  }

  // ---- load ----
  if constexpr (MODE == ROWS_FWD) {
    const float* x = (const float*)in;
    for (int e = tid; e < B * L; e += NT) lds[e] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int e = tid; e < B * n; e += NT) {
      const int b = e / n, c = e - b * n;
      const int r = seq0 + b;
      const float val = x[(size_t)r * n + c] * deapod[r] * deapod[c];
      lds[slot<L>(b, (c - half) & (L - 1))] = make_float2(val, 0.f);
    }
  } else if constexpr (MODE == COLS_FWD || MODE == COLS_TOEP) {
    const float2* h = (const float2*)in;
    for (int e = tid; e < B * L; e += NT) lds[e] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int e = tid; e < B * n; e += NT) {
      const int r = e / B, b = e - r * B;
      lds[slot<L>(b, (r - half) & (L - 1))] = h[(size_t)r * K + seq0 + b];
    }
  } else if constexpr (MODE == COLS_ADJ || MODE == FULL_COLS) {
    const float2* g = (const float2*)in;
    for (int e = tid; e < B * L; e += NT) {
      const int r = e / B, b = e - r * B;
      lds[slot<L>(b, r)] = g[(size_t)r * K + seq0 + b];
    }
  } else if constexpr (MODE == ROWS_ADJ_H) {
    const float2* h = (const float2*)in;
    for (int e = tid; e < B * L; e += NT) {
      const int b = e / L, c = e - b * L;
      const float2* row = h + (size_t)(seq0 + b) * K;
      if (c <= L / 2) {
        lds[slot<L>(b, c)] = row[c];
      } else {
        const float2 v = row[L - c];
        lds[slot<L>(b, c)] = make_float2(v.x, -v.y);
      }
    }
  } else {  // ROWS_ADJ, FULL_ROWS
    const float2* h = (const float2*)in;
    for (int e = tid; e < B * L; e += NT) {
      const int b = e / L, c = e - b * L;
      lds[slot<L>(b, c)] = h[(size_t)(seq0 + b) * K + c];
    }
  }
  __syncthreads();

  // ---- transform: thread tid works on sequence tid / (L/8) ----
  const int sq = tid / (L / 8), lt = tid % (L / 8);
  fft_lds<L, INV>(lds + sq * L, tw, lt, (sq & 3) << 2);
  if constexpr (MODE == COLS_TOEP) {
    // lds[b L + k] *= Ht[(seq0 + b) K + k]: column seq0 + b of the spectrum, read contiguously
    for (int e = tid; e < B * L; e += NT) {
      const float hv = deapod[(size_t)seq0 * K + e];
      const int o = slot<L>(e / L, e % L);
      const float2 v = lds[o];
      lds[o] = make_float2(v.x * hv, v.y * hv);
    }
    __syncthreads();
    fft_lds<L, true>(lds + sq * L, tw, lt, (sq & 3) << 2);
  }

  // ---- store ----
  if constexpr (MODE == ROWS_FWD) {
    float2* h = (float2*)out;
    for (int e = tid; e < B * L; e += NT) {
      const int b = e / L, k = e - b * L;
      h[(size_t)(seq0 + b) * K + k] = lds[slot<L>(b, k)];
    }
  } else if constexpr (MODE == COLS_FWD || MODE == FULL_COLS) {
    float2* g = (float2*)out;
    for (int e = tid; e < B * L; e += NT) {
      const int k = e / B, b = e - k * B;
      g[(size_t)k * K + seq0 + b] = lds[slot<L>(b, k)];
    }
  } else if constexpr (MODE == FULL_ROWS) {
    float2* h = (float2*)out;
    for (int e = tid; e < B * L; e += NT) {
      const int b = e / L, k = e - b * L;
      h[(size_t)(seq0 + b) * K + k] = lds[slot<L>(b, k)];
    }
  } else if constexpr (MODE == COLS_ADJ || MODE == COLS_TOEP) {
    float2* h = (float2*)out;
    for (int e = tid; e < B * n; e += NT) {
      const int r = e / B, b = e - r * B;
      h[(size_t)r * K + seq0 + b] = lds[slot<L>(b, (r - half) & (L - 1))];
    }
  } else {  // ROWS_ADJ, ROWS_ADJ_H
    float* x = (float*)out;
    for (int e = tid; e < B * n; e += NT) {
      const int b = e / n, c = e - b * n;
      const int r = seq0 + b;
      x[(size_t)r * n + c] = lds[slot<L>(b, (c - half) & (L - 1))].x * deapod[r] * deapod[c];
    }
  }
}

template <int L, int MODE>
sh_status launch_len(int per, int P, const void* in, void* out, const float2* tw, const float* deapod, int n,
                     hipStream_t st) {
  constexpr int B = (8192 / L) < 1 ? 1 : (8192 / L);
  int b = B > 64 ? 64 : B;
  while (b > per) b >>= 1;  // few sequences (tiny images): shrink the batch
  // Shrink the batch (down to one wave per work-group) while the pass has fewer than two work-groups per
  // CU, so that more CUs share it, and further up to eight per CU, which hides more of each
  // work-group's load-transform-store latency; a pass that reads or writes columns of a row-major array
  // stops at four columns (32 contiguous bytes of each row) once it has two work-groups per CU, since
  // narrower column reads cost more than the extra work-groups gain.
  constexpr bool STRIDED = MODE == COLS_FWD || MODE == COLS_ADJ || MODE == COLS_TOEP || MODE == FULL_COLS;
  auto groups = [&](int bb) { return int64_t(P) * (per / bb); };
  while (b > 1 && (b / 2) * L / 8 >= 64 &&
         (groups(b) < 512 || (groups(b) < 2048 && (!STRIDED || b / 2 >= 4))))
    b >>= 1;
  const size_t lds = size_t(b) * L * sizeof(float2);
#define SH_FFT_CASE(BB)                                                                                  \
  if (b == BB) {                                                                                         \
    hipLaunchKernelGGL((fft_pass<L, BB, MODE>), dim3(P * (per / BB)), dim3(BB * L / 8), lds, st, in, out, \
                       tw, deapod, n, per);                                                              \
    SH_LAUNCHED();                                                                                       \
    return SH_OK;                                                                                        \
  }
  if constexpr (B >= 64) SH_FFT_CASE(64)
  if constexpr (B >= 32) SH_FFT_CASE(32)
  if constexpr (B >= 16) SH_FFT_CASE(16)
  if constexpr (B >= 8) SH_FFT_CASE(8)
  if constexpr (B >= 4) SH_FFT_CASE(4)
  if constexpr (B >= 2) SH_FFT_CASE(2)
  SH_FFT_CASE(1)
#undef SH_FFT_CASE
  sh::set_error("fft batch size");
  return SH_EUNSUPPORTED;
}

template <int MODE>
sh_status launch_mode(int L, int per, int P, const void* in, void* out, const float2* tw, const float* deapod, int n,
                      hipStream_t st) {
  switch (L) {
    case 32: return launch_len<32, MODE>(per, P, in, out, tw, deapod, n, st);
    case 64: return launch_len<64, MODE>(per, P, in, out, tw, deapod, n, st);
    case 128: return launch_len<128, MODE>(per, P, in, out, tw, deapod, n, st);
    case 256: return launch_len<256, MODE>(per, P, in, out, tw, deapod, n, st);
    case 512: return launch_len<512, MODE>(per, P, in, out, tw, deapod, n, st);
    case 1024: return launch_len<1024, MODE>(per, P, in, out, tw, deapod, n, st);
    case 2048: return launch_len<2048, MODE>(per, P, in, out, tw, deapod, n, st);
    case 4096: return launch_len<4096, MODE>(per, P, in, out, tw, deapod, n, st);
    case 8192: return launch_len<8192, MODE>(per, P, in, out, tw, deapod, n, st);
  }
  sh::set_error("unsupported FFT length %d", L);
  return SH_EUNSUPPORTED;
}

}  // namespace

namespace sh {

sh_status fft_forward_2d(sh_op op, const float* x, float2* grid, hipStream_t st) {
  {
    ProfScope ps("fft_rows", st);
    SH_TRY(launch_mode<ROWS_FWD>(op->K, op->n, op->P, x, op->half.ptr, op->tw.ptr, op->deapod.ptr, op->n, st));
  }
  ProfScope ps("fft_cols", st);
  return launch_mode<COLS_FWD>(op->K, op->K, op->P, op->half.ptr, grid, op->tw.ptr, op->deapod.ptr, op->n, st);
}

sh_status fft_adjoint_2d(sh_op op, const float2* grid, float* x, hipStream_t st) {
  {
    ProfScope ps("fft_cols", st);
    SH_TRY(launch_mode<COLS_ADJ>(op->K, op->K, op->P, grid, op->half.ptr, op->tw.ptr, op->deapod.ptr, op->n, st));
  }
  ProfScope ps("fft_rows", st);
  return launch_mode<ROWS_ADJ>(op->K, op->n, op->P, op->half.ptr, x, op->tw.ptr, op->deapod.ptr, op->n, st);
}

sh_status fft_full_2d(sh_op op, float2* buf, float2* tmp, hipStream_t st) {
  SH_TRY(launch_mode<FULL_ROWS>(op->K, op->K, op->P, buf, tmp, op->tw.ptr, op->ones.ptr, op->n, st));
  return launch_mode<FULL_COLS>(op->K, op->K, op->P, tmp, buf, op->tw.ptr, op->ones.ptr, op->n, st);
}

// The image is real, so every row of the row pass's output is Hermitian in the column index and so is
// every row after the column pass (the kernel spectrum is real and even): the column pass runs over
// columns 0..K/2 only (rounded up to whole work-groups) and the last row pass mirrors the rest.
sh_status toeplitz_apply(sh_op op, const float* Ht, const float* x, float2* tq, float* out, hipStream_t st) {
  ProfScope ps("toeplitz", st);
  const int K = op->K;
  const int b0 = std::min(8192 / K, 64);                 // the column pass's work-group batch (launch_len)
  const int cols = std::min<int>(K, int(cdiv(K / 2 + 1, b0) * b0));
  SH_TRY(launch_mode<ROWS_FWD>(K, op->n, op->P, x, op->half.ptr, op->tw.ptr, op->ones.ptr, op->n, st));
  SH_TRY(launch_mode<COLS_TOEP>(K, cols, op->P, op->half.ptr, tq, op->tw.ptr, Ht, op->n, st));
  return launch_mode<ROWS_ADJ_H>(K, op->n, op->P, tq, out, op->tw.ptr, op->ones.ptr, op->n, st);
}

}  // namespace sh
