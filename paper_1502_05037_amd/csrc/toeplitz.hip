// Toeplitz form of the real normal operator Re(Phi^H Phi) used by the x-update (Q in the SDMM
// paragraph; Phi from the discretised measurement equation).
//
// For the measurement model (Phi x)_m = sum_p x_p exp(-i u_m . (p - n/2)), the real normal operator
// is a 2D convolution of the image with the real kernel
//     k(d) = Re sum_m exp(i u_m . d),   d in (-n, n)^2,
// so it is applied exactly as a circulant on any grid of side K >= 2n - 1: zero-pad, forward DFT,
// multiply by the DFT of the circularly embedded kernel, inverse DFT, crop.  The NUFFT grid side
// K = alpha n (alpha >= 2) is such a grid, and its FFT passes without deapodisation do the padding,
// the transforms and the crop.
//
// The kernel is computed once per plan with the operator's own adjoint: for a shift c,
// Re Phi^H w with w_m = exp(i u_m . c) is k(d) over the window d in [c - n/2, c + n/2)^2, and the
// four shifts c in {-n/2, +n/2}^2 cover d in [-n, n)^2.  With per-block weights a_b the same steps give
// sum_b a_b^2 Re(Phi_b^H Phi_b) (each visibility's modulated unit value carries a_b^2).  u_m is the plan's
// fixed-point coordinate
// (the one the interpolation uses), so the Toeplitz operator agrees with the NUFFT pair to the
// interpolation's accuracy.  The embedded kernel is symmetric up to rounding; the real part of its
// DFT is kept (the DFT of its symmetric part).
#include <cmath>
#include <memory>

#include "op.hpp"

namespace {

// w_m = a_b exp(i u_m . c) with u = 2 pi kappa / K, kappa = cell + fraction from the packed coordinate,
// a_b the weight of the visibility's block (1 without wblk); one work-group per reduction chunk (chunks
// never straddle a block).  The phase is reduced mod K in float64 before the sine and cosine; since
// c is an integer, the wrap of the cell index mod K does not change it.
__global__ __launch_bounds__(256) void modulate_kernel(const uint2* __restrict__ coord, const int4* __restrict__ chunks,
                                                       const float* __restrict__ wblk, float2* __restrict__ w,
                                                       int log2K, int c1, int c2) {
  const int4 ch = chunks[blockIdx.x];
  const float a = wblk ? wblk[ch.x] : 1.0f;
  const int F = 32 - log2K;
  const uint32_t fmask = (1u << F) - 1u;
  const double K = double(1 << log2K);
  for (int i = ch.y + threadIdx.x; i < ch.z; i += 256) {
    const uint2 q = coord[i];
    const double k1 = double(q.x >> F) + ldexp(double(q.x & fmask), -F);
    const double k2 = double(q.y >> F) + ldexp(double(q.y & fmask), -F);
    const double t = k1 * c1 + k2 * c2;
    const double r = t - K * floor(t / K);
    double s, c;
    sincos(2.0 * M_PI * r / K, &s, &c);
    w[i] = make_float2(a * float(c), a * float(s));
  }
}

// Ht[p] *= f[p]
__global__ void scale_spectrum(float* __restrict__ Ht, int64_t KK, const float* __restrict__ f) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < KK) Ht[(size_t)blockIdx.y * KK + j] *= f[blockIdx.y];
}

// Window pixel (r, c) holds k(r + o1, c + o2); it goes to C[(r + o1) mod K][(c + o2) mod K].
__global__ void place_window(const float* __restrict__ win, float2* __restrict__ C, int n, int log2K, int o1,
                             int o2) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (j >= nn) return;
  const int p = blockIdx.y;
  const int K = 1 << log2K;
  const int r = int(j / n), c = int(j - (int64_t)r * n);
  const size_t at = ((size_t)p << (2 * log2K)) + (size_t)((r + o1) & (K - 1)) * K + ((c + o2) & (K - 1));
  C[at] = make_float2(win[(size_t)p * nn + j], 0.f);
}

// Ht[p][k2][k1] = Re spec[p][k1][k2] * scale[p] / K^2
__global__ void spectrum_transpose(const float2* __restrict__ spec, float* __restrict__ Ht, int log2K,
                                   const float* __restrict__ scale) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t KK = int64_t(1) << (2 * log2K);
  if (j >= KK) return;
  const int p = blockIdx.y;
  const int K = 1 << log2K;
  const int k1 = int(j >> log2K), k2 = int(j & (K - 1));
  Ht[(size_t)p * KK + (size_t)k2 * K + k1] = spec[(size_t)p * KK + j].x * scale[p];
}

}  // namespace

namespace sh {

sh_status toeplitz_build(sh_op op, const double* scale, const double* wblk, sh_toep_s* t, hipStream_t st) {
  const int n = op->n, K = op->K, P = op->P;
  SH_REQUIRE(K >= 2 * n, "the Toeplitz embedding needs a grid side K >= 2n (K = %d, n = %d)", K, n);
  const int64_t M = op->M, nn = (int64_t)n * n, KK = (int64_t)K * K;
  std::vector<float> sc(P);
  for (int p = 0; p < P; ++p) {
    const double v = scale ? scale[p] : 1.0;
    SH_REQUIRE(std::isfinite(v) && v > 0, "scale[%d] must be positive and finite, got %g", p, v);
    sc[p] = float(v / (double(K) * double(K)));
  }
  // the operator's own arrays first, the build's temporaries after them (so that a workspace arena can
  // take the temporaries back when they are released)
  SH_TRY(t->Ht.alloc(P * KK));
  SH_TRY(t->tq.alloc((int64_t)P * n * K));
  if (!op->ones.ptr) {   // the FFT passes' unit weights belong to the plan: never from a caller's workspace
    sh::ArenaScope none(nullptr);
    SH_TRY(op->ones.upload(std::vector<float>(n, 1.0f)));
  }
  sh::DevBuf<float2> w, C, tmp;
  sh::DevBuf<float> win, scd, wb;
  if (wblk) {   // a visibility of block b carries wblk[b]^2: the modulated vector and the adjoint's weight
    std::vector<float> a(op->R);
    for (int i = 0; i < op->R; ++i) {
      SH_REQUIRE(std::isfinite(wblk[i]) && wblk[i] > 0, "block weight %d must be positive and finite", i);
      a[i] = float(wblk[i] * wblk[i]);
    }
    SH_TRY(wb.upload(a));
  }
  SH_TRY(w.alloc(M));
  SH_TRY(win.alloc(P * nn));
  SH_TRY(C.alloc(P * KK));
  SH_TRY(tmp.alloc(P * KK));
  SH_TRY(scd.upload(sc));
  SH_HIP(hipMemsetAsync(C.ptr, 0, P * KK * sizeof(float2), st));
  for (int s1 = 0; s1 < 2; ++s1)
    for (int s2 = 0; s2 < 2; ++s2) {
      const int c1 = s1 ? n / 2 : -n / 2, c2 = s2 ? n / 2 : -n / 2;
      hipLaunchKernelGGL(modulate_kernel, dim3((unsigned)op->n_chunks), dim3(256), 0, st, op->coord.ptr,
                         op->chunks.ptr, wblk ? wb.ptr : nullptr, w.ptr, op->log2K, c1, c2);
      SH_LAUNCHED();
      SH_TRY(phi_adjoint(op, w.ptr, win.ptr, false, nullptr, st));
      hipLaunchKernelGGL(place_window, dim3((unsigned)cdiv(nn, 256), P), dim3(256), 0, st, win.ptr, C.ptr, n,
                         op->log2K, c1 - n / 2, c2 - n / 2);
      SH_LAUNCHED();
    }
  SH_TRY(fft_full_2d(op, C.ptr, tmp.ptr, st));
  hipLaunchKernelGGL(spectrum_transpose, dim3((unsigned)cdiv(KK, 256), P), dim3(256), 0, st, C.ptr, t->Ht.ptr,
                     op->log2K, scd.ptr);
  SH_LAUNCHED();
  t->op = op;
  // the temporaries are freed on return: wait for the kernels that read them
  SH_HIP(hipStreamSynchronize(st));
  return SH_OK;
}

sh_status toeplitz_rescale(sh_toep_s* t, const double* factor, hipStream_t st) {
  sh_op op = t->op;
  const int P = op->P;
  const int64_t KK = int64_t(op->K) * op->K;
  std::vector<float> f(P);
  for (int p = 0; p < P; ++p) f[p] = float(factor[p]);
  sh::DevBuf<float> fd;
  SH_TRY(fd.upload(f));
  hipLaunchKernelGGL(scale_spectrum, dim3((unsigned)cdiv(KK, 256), P), dim3(256), 0, st, t->Ht.ptr, KK, fd.ptr);
  SH_LAUNCHED();
  SH_HIP(hipStreamSynchronize(st));   // fd is freed on return
  return SH_OK;
}

}  // namespace sh

extern "C" {

sh_status sh_toeplitz_create(sh_op op, const double* scale, sh_toep* out, void* stream) {
  SH_REQUIRE(op && out, "op and out must be non-NULL");
  *out = nullptr;
  auto t = std::make_unique<sh_toep_s>();
  SH_TRY(sh::toeplitz_build(op, scale, nullptr, t.get(), (hipStream_t)stream));
  *out = t.release();
  return SH_OK;
}

static size_t toeplitz_ws_bytes(sh_op op) {
  using sh::Arena;
  const size_t P = op->P, n = op->n, K = op->K, KK = K * K, M = op->M;
  return Arena::round(4 * P * KK) + Arena::round(8 * P * n * K)                       // spectrum, scratch
         + Arena::round(8 * M) + Arena::round(4 * P * n * n) + 2 * Arena::round(8 * P * KK) + Arena::round(4 * P);
}

sh_status sh_toeplitz_workspace_bytes(sh_op op, size_t* bytes) {
  SH_REQUIRE(op && bytes, "NULL argument");
  *bytes = toeplitz_ws_bytes(op);
  return SH_OK;
}

sh_status sh_toeplitz_create_ws(sh_op op, const double* scale, void* workspace, size_t bytes, sh_toep* out,
                                void* stream) {
  SH_REQUIRE(op && out && workspace, "op, workspace and out must be non-NULL");
  SH_REQUIRE(reinterpret_cast<uintptr_t>(workspace) % sh::Arena::kAlign == 0, "workspace must be %zu-byte aligned",
             sh::Arena::kAlign);
  SH_REQUIRE(bytes >= toeplitz_ws_bytes(op), "workspace of %zu bytes is smaller than the %zu needed", bytes,
             toeplitz_ws_bytes(op));
  *out = nullptr;
  auto t = std::make_unique<sh_toep_s>();
  t->arena.base = static_cast<char*>(workspace);
  t->arena.size = bytes;
  {
    sh::ArenaScope scope(&t->arena);
    SH_TRY(sh::toeplitz_build(op, scale, nullptr, t.get(), (hipStream_t)stream));
  }
  *out = t.release();
  return SH_OK;
}

sh_status sh_toeplitz_apply(sh_toep t, const float* x, float* out, void* stream) {
  SH_REQUIRE(t && x && out, "t, x and out must be non-NULL");
  return sh::toeplitz_apply(t->op, t->Ht.ptr, x, t->tq.ptr, out, (hipStream_t)stream);
}

sh_status sh_toeplitz_destroy(sh_toep t) {
  delete t;
  return SH_OK;
}

}  // extern "C"
