// SARA dictionary Psi = (1/sqrt q) [Dirac, db1, ..., db8] (SARA paragraph: a concatenation of q
// coherent bases, used through Psi^dagger in the analysis prior).
//
// Each Daubechies basis is a 2D periodic orthonormal DWT with `levels` levels in Mallat layout: one
// level filters within rows into [a | d] and then within columns into [a ; d]; quadrants are LL
// (top-left), row-high/column-low (top-right), row-low/column-high (bottom-left), HH (bottom-right).
// Analysis runs one launch per level for all wavelet planes of all images of a batch at once
// (blockIdx.z = image * planes + plane): a
// work-group stages a (2T + 2p - 2)^2 input window in LDS with coalesced row reads, filters along
// rows, then along columns through LDS (the transpose), and writes T x T outputs of each subband.
// Synthesis is the transpose, tile by tile; its last level sums all planes in registers so the
// image is written once.
#include <cmath>

#include "common.hpp"
#include "tables.hpp"

struct DwtPlanes {
  int nplanes;        // wavelet planes (Dirac excluded)
  int dirac_plane;    // coefficient plane of the Dirac basis, or -1
  int plane[8];       // coefficient plane of wavelet plane d
  int flen[8];        // 2p
  float h[8][16];
  float g[8][16];
};

struct sh_psi_s {
  int n = 0, levels = 0, q = 0;
  int batch = 1;                  // images transformed per call (image-major: x[img][n][n], c[img][q][n][n])
  uint32_t mask = 0;
  float scale = 1.f;
  DwtPlanes pl{};
  sh::Arena arena;                // a caller's workspace (sh_psi_create_ws); declared before the buffers
  sh::DevBuf<float> tmpA, tmpB;   // batch x nplanes x (n/2)^2 LL ping-pong
};

namespace {

constexpr int AT = 16;                 // analysis output tile (subband coordinates)
constexpr int AIN = 2 * AT + 16 - 2;   // input window side for filters up to 16 taps
constexpr int ST = 32;                 // synthesis output tile
constexpr int SK = ST / 2 + 8;         // subband window side

// One analysis level.  Input: side L (ld in_ld, plane stride in_ps, 0 = shared by the planes of an
// image; image stride in_is), scaled by `s0`.  Details go to coefficient planes (ld n, image stride
// c_is); LL goes to ll_out (ld ll_ld, plane stride ll_ps, image stride nplanes * ll_ps) or, if ll_out
// is NULL, to the top-left of the coefficient plane.
__global__ __launch_bounds__(256) void dwt_analysis(const float* __restrict__ in, int in_ld, int64_t in_ps,
                                                    int64_t in_is, int L, float* __restrict__ coeffs, int n,
                                                    int64_t c_is, float* __restrict__ ll_out, int ll_ld, int64_t ll_ps,
                                                    float s0, DwtPlanes pl) {
  __shared__ float win[AIN][AIN + 1];
  __shared__ float ra[AIN][AT + 1];
  __shared__ float rd[AIN][AT + 1];
  const int img = blockIdx.z / pl.nplanes;
  const int d = blockIdx.z - img * pl.nplanes;
  in += img * in_is;
  coeffs += img * c_is;
  if (ll_out) ll_out += (int64_t)img * pl.nplanes * ll_ps;
  const int Lf = pl.flen[d];
  const int H = L / 2;
  const int te = H < AT ? H : AT;          // effective tile side
  const int k1_0 = blockIdx.y * te, k2_0 = blockIdx.x * te;
  const int nin = 2 * te + Lf - 2;
  const float* src = in + (int64_t)d * in_ps;
  const int tid = threadIdx.x;
  for (int e = tid; e < nin * nin; e += 256) {
    const int r = e / nin, c = e - r * nin;
    const int gr = (2 * k1_0 + r) % L, gc = (2 * k2_0 + c) % L;
    win[r][c] = src[(int64_t)gr * in_ld + gc] * s0;
  }
  __syncthreads();
  // rows: a/d for every window row and each output column of the tile
  for (int e = tid; e < nin * te; e += 256) {
    const int r = e / te, k = e - r * te;
    float a = 0.f, dd = 0.f;
    for (int t = 0; t < Lf; ++t) {
      const float v = win[r][2 * k + t];
      a = fmaf(pl.h[d][t], v, a);
      dd = fmaf(pl.g[d][t], v, dd);
    }
    ra[r][k] = a;
    rd[r][k] = dd;
  }
  __syncthreads();
  float* plane = coeffs + (int64_t)pl.plane[d] * n * n;
  for (int e = tid; e < te * te; e += 256) {
    const int k1 = e / te, k2 = e - k1 * te;
    float ll = 0.f, lh = 0.f, hl = 0.f, hh = 0.f;
    for (int t = 0; t < Lf; ++t) {
      const float va = ra[2 * k1 + t][k2], vd = rd[2 * k1 + t][k2];
      ll = fmaf(pl.h[d][t], va, ll);
      lh = fmaf(pl.g[d][t], va, lh);   // row-low, column-high
      hl = fmaf(pl.h[d][t], vd, hl);   // row-high, column-low
      hh = fmaf(pl.g[d][t], vd, hh);
    }
    const int o1 = k1_0 + k1, o2 = k2_0 + k2;
    if (o1 >= H || o2 >= H) continue;
    plane[(int64_t)o1 * n + H + o2] = hl;
    plane[(int64_t)(H + o1) * n + o2] = lh;
    plane[(int64_t)(H + o1) * n + H + o2] = hh;
    if (ll_out)
      ll_out[(int64_t)d * ll_ps + (int64_t)o1 * ll_ld + o2] = ll;
    else
      plane[(int64_t)o1 * n + o2] = ll;
  }
}

// One synthesis level producing side L from subbands of side H = L/2.  LL comes from ll_in (ld
// ll_ld, plane stride ll_ps, image stride nplanes * ll_ps) or, if NULL, from the coefficient plane
// (image stride c_is).  If `sum_out` is set, work-group z (= image) loops over all wavelet planes,
// adds the Dirac plane and writes s_out * sum to `out` (ld n, image stride n^2); otherwise
// z = image * nplanes + plane goes to out + z * out_ps (ld out_ld).
__global__ __launch_bounds__(256) void dwt_synthesis(const float* __restrict__ ll_in, int ll_ld, int64_t ll_ps, int L,
                                                     const float* __restrict__ coeffs, int n, int64_t c_is,
                                                     float* __restrict__ out, int out_ld, int64_t out_ps, int sum_out,
                                                     float s_out, DwtPlanes pl) {
  __shared__ float sb[4][SK][SK + 1];    // LL, HL, LH, HH windows
  __shared__ float ylo[ST][SK + 1];      // column-synthesised, row-low half
  __shared__ float yhi[ST][SK + 1];      // column-synthesised, row-high half
  const int H = L / 2;
  const int te = L < ST ? L : ST;
  const int i0 = blockIdx.y * te, j0 = blockIdx.x * te;
  const int tid = threadIdx.x;
  float acc[ST * ST / 256];
#pragma unroll
  for (int q = 0; q < ST * ST / 256; ++q) acc[q] = 0.f;
  const int img = sum_out ? (int)blockIdx.z : (int)blockIdx.z / pl.nplanes;
  const int d_begin = sum_out ? 0 : blockIdx.z - img * pl.nplanes;
  const int d_end = sum_out ? pl.nplanes : d_begin + 1;
  coeffs += img * c_is;
  if (ll_in) ll_in += (int64_t)img * pl.nplanes * ll_ps;
  for (int d = d_begin; d < d_end; ++d) {
    const int Lf = pl.flen[d];
    const int kw = te / 2 + Lf / 2 - 1;                  // window side in subband coordinates
    const int kr0 = i0 / 2 - Lf / 2 + 1, kc0 = j0 / 2 - Lf / 2 + 1;
    const float* plane = coeffs + (int64_t)pl.plane[d] * n * n;
    const float* llp = ll_in ? ll_in + (int64_t)d * ll_ps : plane;
    const int lld = ll_in ? ll_ld : n;
    __syncthreads();
    for (int e = tid; e < kw * kw; e += 256) {
      const int r = e / kw, c = e - r * kw;
      const int kr = ((kr0 + r) % H + H) % H, kc = ((kc0 + c) % H + H) % H;
      sb[0][r][c] = llp[(int64_t)kr * lld + kc];
      sb[1][r][c] = plane[(int64_t)kr * n + H + kc];
      sb[2][r][c] = plane[(int64_t)(H + kr) * n + kc];
      sb[3][r][c] = plane[(int64_t)(H + kr) * n + H + kc];
    }
    __syncthreads();
    // columns: y[i][c] = sum_t [i - t even] (h[t] top[k][c] + g[t] bottom[k][c]), k = ((i - t) mod L) / 2.
    // Window row r holds subband row (kr0 + r) mod H, so k is window row (i - t)/2 + Lf/2 - 1 (local
    // i; i0 is even), which lies in [0, kw) for every tap: no modulo in the loop.
    for (int e = tid; e < te * kw; e += 256) {
      const int i = e / kw, c = e - i * kw;
      const int gi = i0 + i;
      float lo = 0.f, hi = 0.f;
      for (int t = (gi & 1); t < Lf; t += 2) {
        const int r = ((i - t) >> 1) + Lf / 2 - 1;       // window row of subband row ((gi - t) mod L) / 2
        lo = fmaf(pl.h[d][t], sb[0][r][c], lo);
        lo = fmaf(pl.g[d][t], sb[2][r][c], lo);
        hi = fmaf(pl.h[d][t], sb[1][r][c], hi);
        hi = fmaf(pl.g[d][t], sb[3][r][c], hi);
      }
      ylo[i][c] = lo;
      yhi[i][c] = hi;
    }
    __syncthreads();
    // rows: x[i][j] = sum_t [j - t even] (h[t] ylo[i][c] + g[t] yhi[i][c]), c = ((j - t) mod L) / 2
    for (int q = 0; q < ST * ST / 256; ++q) {
      const int e = tid + q * 256;
      const int i = e / ST, j = e - i * ST;
      if (i >= te || j >= te) continue;
      const int gj = j0 + j;
      float v = 0.f;
      for (int t = (gj & 1); t < Lf; t += 2) {
        const int c = ((j - t) >> 1) + Lf / 2 - 1;       // window column, as for the rows above
        v = fmaf(pl.h[d][t], ylo[i][c], v);
        v = fmaf(pl.g[d][t], yhi[i][c], v);
      }
      acc[q] += v;
    }
  }
  for (int q = 0; q < ST * ST / 256; ++q) {
    const int e = tid + q * 256;
    const int i = e / ST, j = e - i * ST;
    if (i >= te || j >= te) continue;
    const int gi = i0 + i, gj = j0 + j;
    if (gi >= L || gj >= L) continue;
    if (sum_out) {
      float v = acc[q];
      if (pl.dirac_plane >= 0) v += coeffs[(int64_t)pl.dirac_plane * n * n + (int64_t)gi * n + gj];
      out[(int64_t)img * n * n + (int64_t)gi * n + gj] = v * s_out;
    } else {
      out[(int64_t)blockIdx.z * out_ps + (int64_t)gi * out_ld + gj] = acc[q];
    }
  }
}

// Dirac plane: y[img * ys + i] = s * x[img * xs + i], i < N, img = blockIdx.y.
__global__ void scale_copy(const float* __restrict__ x, int64_t xs, float* __restrict__ y, int64_t ys, int64_t N,
                           float s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) y[blockIdx.y * ys + i] = x[blockIdx.y * xs + i] * s;
}

}  // namespace

extern "C" {

sh_status sh_daubechies(int32_t p, double* h_out) {
  SH_REQUIRE(h_out && p >= 1 && p <= 8, "p must be in [1, 8]");
  if (!sh::daubechies(p, h_out)) {
    sh::set_error("daubechies(%d) failed", p);
    return SH_EUNSUPPORTED;
  }
  return SH_OK;
}

static int wavelet_planes(uint32_t basis_mask) {
  int k = 0;
  for (int b = 1; b < 9; ++b) k += (basis_mask >> b) & 1;
  return k;
}

static size_t psi_ws_bytes(int32_t n, uint32_t basis_mask, int32_t batch) {
  const size_t half = size_t(n / 2) * (n / 2) * wavelet_planes(basis_mask) * batch * sizeof(float);
  return half ? 2 * sh::Arena::round(half) : 0;
}

static sh_status psi_create(int32_t n, int32_t levels, uint32_t basis_mask, int32_t batch, void* workspace,
                            size_t bytes, sh_psi* out);

extern "C" sh_status sh_psi_workspace_bytes(int32_t n, int32_t levels, uint32_t basis_mask, int32_t batch,
                                            size_t* bytes) {
  SH_REQUIRE(bytes, "bytes is NULL");
  SH_REQUIRE(batch >= 1 && batch <= 4096 && n >= 2 && basis_mask != 0 && (basis_mask >> 9) == 0 && levels >= 1,
             "invalid dictionary");
  *bytes = psi_ws_bytes(n, basis_mask, batch);
  return SH_OK;
}

extern "C" sh_status sh_psi_create_ws(int32_t n, int32_t levels, uint32_t basis_mask, int32_t batch, void* workspace,
                                      size_t bytes, sh_psi* out) {
  SH_REQUIRE(workspace || psi_ws_bytes(n, basis_mask, batch) == 0, "workspace is NULL");
  SH_REQUIRE(reinterpret_cast<uintptr_t>(workspace) % sh::Arena::kAlign == 0, "workspace must be %zu-byte aligned",
             sh::Arena::kAlign);
  SH_REQUIRE(bytes >= psi_ws_bytes(n, basis_mask, batch), "workspace of %zu bytes is smaller than the %zu needed",
             bytes, psi_ws_bytes(n, basis_mask, batch));
  return psi_create(n, levels, basis_mask, batch, workspace, bytes, out);
}

sh_status sh_psi_create_batched(int32_t n, int32_t levels, uint32_t basis_mask, int32_t batch, sh_psi* out) {
  return psi_create(n, levels, basis_mask, batch, nullptr, 0, out);
}

static sh_status psi_create(int32_t n, int32_t levels, uint32_t basis_mask, int32_t batch, void* workspace,
                            size_t bytes, sh_psi* out) {
  SH_REQUIRE(out, "out is NULL");
  *out = nullptr;
  SH_REQUIRE(batch >= 1 && batch <= 4096, "batch must be in [1, 4096]");
  SH_REQUIRE(levels >= 1 && levels <= 8, "levels must be in [1, 8]");
  SH_REQUIRE(n >= 2 && n <= 8192 && n % (1 << levels) == 0, "n = %d must be divisible by 2^levels", n);
  SH_REQUIRE(basis_mask != 0 && (basis_mask >> 9) == 0, "basis mask must be a non-empty subset of 0x1FF");
  sh_psi psi = new (std::nothrow) sh_psi_s();
  if (!psi) {
    sh::set_error("host allocation failed");
    return SH_ENOMEM;
  }
  psi->n = n;
  psi->batch = batch;
  psi->levels = levels;
  psi->mask = basis_mask;
  int plane = 0;
  psi->pl.dirac_plane = -1;
  for (int b = 0; b < 9; ++b) {
    if (!(basis_mask >> b & 1)) continue;
    if (b == 0) {
      psi->pl.dirac_plane = plane++;
      continue;
    }
    const int d = psi->pl.nplanes++;
    psi->pl.plane[d] = plane++;
    psi->pl.flen[d] = 2 * b;
    double h[16];
    sh::daubechies(b, h);
    for (int t = 0; t < 16; ++t) {
      psi->pl.h[d][t] = t < 2 * b ? float(h[t]) : 0.f;
      psi->pl.g[d][t] = t < 2 * b ? float((t % 2 ? -1.0 : 1.0) * h[2 * b - 1 - t]) : 0.f;
    }
  }
  psi->q = plane;
  psi->scale = float(1.0 / std::sqrt(double(plane)));
  if (psi->pl.nplanes > 0) {
    const size_t half = size_t(n / 2) * (n / 2) * psi->pl.nplanes * batch;
    psi->arena.base = static_cast<char*>(workspace);
    psi->arena.size = bytes;
    sh::ArenaScope scope(workspace ? &psi->arena : nullptr);
    sh_status s = psi->tmpA.alloc(half);
    if (s == SH_OK) s = psi->tmpB.alloc(half);
    if (s != SH_OK) {
      delete psi;
      return s;
    }
  }
  *out = psi;
  return SH_OK;
}

sh_status sh_psi_create(int32_t n, int32_t levels, uint32_t basis_mask, sh_psi* out) {
  return sh_psi_create_batched(n, levels, basis_mask, 1, out);
}

sh_status sh_psi_destroy(sh_psi psi) {
  delete psi;
  return SH_OK;
}

sh_status sh_psi_planes(sh_psi psi, int32_t* q_out) {
  SH_REQUIRE(psi && q_out, "NULL argument");
  *q_out = psi->q;
  return SH_OK;
}

sh_status sh_psi_adj(sh_psi psi, const float* x, float* coeffs, void* stream) {
  SH_REQUIRE(psi && x && coeffs, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const int n = psi->n, B = psi->batch;
  const int64_t N = int64_t(n) * n, c_is = int64_t(psi->q) * N;
  sh::ProfScope ps("dwt", st);
  if (psi->pl.dirac_plane >= 0) {
    hipLaunchKernelGGL(scale_copy, dim3((unsigned)sh::cdiv(N, 256), B), dim3(256), 0, st, x, N,
                       coeffs + (int64_t)psi->pl.dirac_plane * N, c_is, N, psi->scale);
    SH_LAUNCHED();
  }
  const int np = psi->pl.nplanes;
  if (np == 0) return SH_OK;
  const float* in = x;
  int in_ld = n;
  int64_t in_ps = 0, in_is = N;
  float s0 = psi->scale;
  float* bufs[2] = {psi->tmpA.ptr, psi->tmpB.ptr};
  for (int lev = 0; lev < psi->levels; ++lev) {
    const int L = n >> lev, H = L / 2;
    const int te = H < AT ? H : AT;
    const bool last = lev == psi->levels - 1;
    float* llo = last ? nullptr : bufs[lev & 1];
    const unsigned nt = (unsigned)sh::cdiv(H, te);
    dim3 grid(nt, nt, np * B);
    hipLaunchKernelGGL(dwt_analysis, grid, dim3(256), 0, st, in, in_ld, in_ps, in_is, L, coeffs, n, c_is, llo, H,
                       int64_t(H) * H, s0, psi->pl);
    SH_LAUNCHED();
    in = llo;
    in_ld = H;
    in_ps = int64_t(H) * H;
    in_is = in_ps * np;
    s0 = 1.f;
  }
  return SH_OK;
}

sh_status sh_psi_fwd(sh_psi psi, const float* coeffs, float* x, void* stream) {
  SH_REQUIRE(psi && x && coeffs, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const int n = psi->n, B = psi->batch;
  const int64_t N = int64_t(n) * n, c_is = int64_t(psi->q) * N;
  sh::ProfScope ps("dwt", st);
  const int np = psi->pl.nplanes;
  if (np == 0) {  // Dirac only
    hipLaunchKernelGGL(scale_copy, dim3((unsigned)sh::cdiv(N, 256), B), dim3(256), 0, st,
                       coeffs + (int64_t)psi->pl.dirac_plane * N, c_is, x, N, N, psi->scale);
    SH_LAUNCHED();
    return SH_OK;
  }
  float* bufs[2] = {psi->tmpA.ptr, psi->tmpB.ptr};
  const float* ll = nullptr;  // coarsest LL lives in the coefficient plane
  int ll_ld = n;
  int64_t ll_ps = 0;
  for (int lev = psi->levels - 1; lev >= 0; --lev) {
    const int L = n >> lev;
    const int te = L < ST ? L : ST;
    const unsigned nt = (unsigned)sh::cdiv(L, te);
    if (lev > 0) {
      float* o = bufs[lev & 1];
      dim3 grid(nt, nt, np * B);
      hipLaunchKernelGGL(dwt_synthesis, grid, dim3(256), 0, st, ll, ll_ld, ll_ps, L, coeffs, n, c_is, o, L,
                         int64_t(L) * L, 0, 1.f, psi->pl);
      SH_LAUNCHED();
      ll = o;
      ll_ld = L;
      ll_ps = int64_t(L) * L;
    } else {
      dim3 grid(nt, nt, B);
      hipLaunchKernelGGL(dwt_synthesis, grid, dim3(256), 0, st, ll, ll_ld, ll_ps, L, coeffs, n, c_is, x, n, 0, 1,
                         psi->scale, psi->pl);
      SH_LAUNCHED();
    }
  }
  return SH_OK;
}

}  // extern "C"

int psi_side(sh_psi psi) { return psi->n; }
int psi_batch(sh_psi psi) { return psi->batch; }
