// Proximal steps of SDMM on problem (3), each fused with its dual update, plus the float64 reductions
// that drive them (per-block l2 norms, CG dot products, the stopping test and the reweighting).
//
// For a split with linear image s = L_j x, dual z and proximal map prox:
//   t = s + z;  y = prox(t);  z <- t - y;  v = y - z   (v feeds the next x-update).
// Reductions are two-stage with a fixed tree (per-work-group partials, then one work-group), so they
// are deterministic.
#include <cmath>
#include <mutex>

#include "prox.hpp"

namespace {

constexpr int RB = 512;   // first-stage work-groups of a one-segment reduction

// Sum of v over the work-group, returned to every thread: a butterfly inside each wave (lane 0's result,
// whose order of additions is fixed), then the waves' sums in wave order.  Two barriers, whatever the size.
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < int(blockDim.x >> 6); ++w) r += sh[w];
  __syncthreads();   // sh is free again for the caller's next sum
  return r;
}

// Sum of part[seg * n, (seg + 1) * n), computed by the whole work-group in the order of sum_final below (so
// that every work-group of a launch, and sum_final, get the same bits), returned to every thread.
__device__ __forceinline__ double seg_total(const double* __restrict__ part, int n, int seg, double* sh) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[(int64_t)seg * n + i];
  return block_sum(acc, sh);
}

// First stages over segments: grid (gridDim.x, P), blockIdx.y = segment; work-group b of segment p
// reduces a grid-stride slice of the segment into part[p * gridDim.x + b].
#define SEGMENT_LOOP(i)                                                                     \
  const int64_t seg0 = (int64_t)blockIdx.y * per;                                           \
  for (int64_t i = seg0 + (int64_t)blockIdx.x * 256 + threadIdx.x; i < seg0 + per; i += (int64_t)gridDim.x * 256)
#define PART_OUT(r) \
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (r)

// Conjugate-gradient steps fused with the dot product that follows them (per segment p = problem):
// r = a + b + c - xc x (c may be NULL), p = r, xprev = x, partial r.r
__global__ __launch_bounds__(256) void cg_init_rr(const float* __restrict__ a, const float* __restrict__ b,
                                                  const float* __restrict__ c, const float* __restrict__ x,
                                                  float* __restrict__ r, float* __restrict__ pv,
                                                  float* __restrict__ xprev, int64_t per, double* __restrict__ part,
                                                  float xc) {
  __shared__ double sh[256];
  double acc = 0.0;
  SEGMENT_LOOP(i) {
    const float xv = x[i];
    const float rv = a[i] + b[i] + (c ? c[i] : 0.f) - xc * xv;
    r[i] = rv;
    pv[i] = rv;
    xprev[i] = xv;
    acc += double(rv) * double(rv);
  }
  const double rs = block_sum(acc, sh);
  PART_OUT(rs);
}

// Ap = pc p + Ap, partial p.Ap
__global__ __launch_bounds__(256) void cg_ap_dot(const float* __restrict__ pv, float* __restrict__ Ap, int64_t per,
                                                 double* __restrict__ part, float pc) {
  __shared__ double sh[256];
  double acc = 0.0;
  SEGMENT_LOOP(i) {
    const float pi = pv[i];
    const float a = pc * pi + Ap[i];
    Ap[i] = a;
    acc += double(pi) * double(a);
  }
  const double r = block_sum(acc, sh);
  PART_OUT(r);
}

// pAp = sum of the p.Ap partials (every work-group; the first of the segment stores it), alpha = rs / pAp;
// x += alpha p; r -= alpha Ap; partial r.r
__global__ __launch_bounds__(256) void cg_update_rr(float* __restrict__ x, float* __restrict__ r,
                                                    const float* __restrict__ pv, const float* __restrict__ Ap,
                                                    int64_t per, const double* __restrict__ rs,
                                                    const double* __restrict__ pap_part, double* __restrict__ pap_out,
                                                    double* __restrict__ part) {
  __shared__ double sh[256];
  const double d = seg_total(pap_part, gridDim.x, blockIdx.y, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) pap_out[blockIdx.y] = d;
  const float alpha = d > 0 ? float(rs[blockIdx.y] / d) : 0.f;
  double acc = 0.0;
  SEGMENT_LOOP(i) {
    x[i] = fmaf(alpha, pv[i], x[i]);
    const float rv = fmaf(-alpha, Ap[i], r[i]);
    r[i] = rv;
    acc += double(rv) * double(rv);
  }
  const double rr = block_sum(acc, sh);
  PART_OUT(rr);
}

// rs_new = sum of the r.r partials (every work-group; the first of the segment stores it), beta = rs_new / rs;
// p = r + beta p
__global__ __launch_bounds__(256) void cg_dir_rr(const float* __restrict__ r, float* __restrict__ pv, int64_t per,
                                                 const double* __restrict__ rs, const double* __restrict__ rr_part,
                                                 double* __restrict__ rs_out) {
  __shared__ double sh[256];
  const double rn = seg_total(rr_part, gridDim.x, blockIdx.y, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) rs_out[blockIdx.y] = rn;
  const double d = rs[blockIdx.y];
  const float beta = d > 0 ? float(rn / d) : 0.f;
  SEGMENT_LOOP(i) pv[i] = fmaf(beta, pv[i], r[i]);
}

// partials of ||x - xprev||^2 (part) and ||x||^2 (part + P * gridDim.x)
__global__ __launch_bounds__(256) void change_dots(const float* __restrict__ x, const float* __restrict__ xprev,
                                                   int64_t per, double* __restrict__ part) {
  __shared__ double sh[256];
  double a = 0.0, b = 0.0;
  SEGMENT_LOOP(i) {
    const float xv = x[i];
    const float d = xv - xprev[i];
    a += double(d) * double(d);
    b += double(xv) * double(xv);
  }
  const double ra = block_sum(a, sh);
  const double rb = block_sum(b, sh);
  PART_OUT(ra);
  if (threadIdx.x == 0) part[(int64_t)gridDim.y * gridDim.x + (int64_t)blockIdx.y * gridDim.x + blockIdx.x] = rb;
}

__global__ __launch_bounds__(256) void dot_partial(const float* __restrict__ a, const float* __restrict__ b, int64_t per,
                                                   double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  SEGMENT_LOOP(i) acc += double(a[i]) * double(b[i]);
  const double r = block_sum(acc, sh);
  PART_OUT(r);
}

// out[p] = sum of part[p*n, (p+1)*n) (work-group p, fixed tree)
__global__ __launch_bounds__(256) void sum_final(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[(int64_t)blockIdx.x * n + i];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void mean_partial(const float* __restrict__ a, int64_t per, double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  SEGMENT_LOOP(i) acc += double(a[i]);
  const double r = block_sum(acc, sh);
  PART_OUT(r);
}

__global__ __launch_bounds__(256) void var_partial(const float* __restrict__ a, int64_t per, const double* __restrict__ sum,
                                                   double* __restrict__ part) {
  __shared__ double sh[256];
  const double mean = sum[blockIdx.y] / double(per);
  double acc = 0.0;
  SEGMENT_LOOP(i) {
    const double d = double(a[i]) - mean;
    acc += d * d;
  }
  const double r = block_sum(acc, sh);
  PART_OUT(r);
}

// Maximum of v over the work-group (for thread 0; exact in any order): per wave, then over the waves.
__device__ __forceinline__ double block_max(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
  for (int w = 1; w < int(blockDim.x >> 6); ++w) r = fmax(r, sh[w]);
  return r;
}

__global__ __launch_bounds__(256) void maxabs_partial(const float* __restrict__ a, int64_t per, double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  SEGMENT_LOOP(i) acc = fmax(acc, fabs(double(a[i])));
  const double r = block_max(acc, sh);
  PART_OUT(r);
}

__global__ __launch_bounds__(256) void max_final(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc = fmax(acc, part[(int64_t)blockIdx.x * n + i]);
  const double r = block_max(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void l1w_partial(const float* __restrict__ c, const float* __restrict__ W, int64_t per,
                                                   double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  SEGMENT_LOOP(i) acc += fabs(double(c[i]) * (W ? double(W[i]) : 1.0));
  const double r = block_sum(acc, sh);
  PART_OUT(r);
}
// partials of sum (a + fb b + fc c)^2 (b, c may be NULL)
__global__ __launch_bounds__(256) void comb3_sq_partial(const float* __restrict__ a, const float* __restrict__ b,
                                                        const float* __restrict__ c, float fb, float fc, int64_t per,
                                                        double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  SEGMENT_LOOP(i) {
    double t = double(a[i]);
    if (b) t += double(fb) * double(b[i]);
    if (c) t += double(fc) * double(c[i]);
    acc += t * t;
  }
  const double r = block_sum(acc, sh);
  PART_OUT(r);
}
#undef SEGMENT_LOOP
#undef PART_OUT

// Primal residual of the data splits (see sdmm.hip: v = cb (y - z - s_hat), s_hat = cb s):
// per-chunk float64 partial sums of ||s_hat - y||^2 = ||v / cb + z||^2 and of ||s_hat||^2
__global__ __launch_bounds__(256) void kkt_vis_partial(const float2* __restrict__ s_in, const float2* __restrict__ z,
                                                       const float2* __restrict__ v, const int4* __restrict__ chunks,
                                                       const float* __restrict__ cblk, double* __restrict__ part,
                                                       int sub_s) {
  __shared__ double sh[256];
  const int4 c = chunks[blockIdx.x];
  const float cb = cblk ? cblk[c.x] : 1.0f;
  double a = 0.0, b = 0.0;
  for (int i = c.y + threadIdx.x; i < c.z; i += 256) {
    const float2 vv = v[i], zv = z[i], sv = s_in[i];
    const double sr = double(cb) * double(sv.x), si = double(cb) * double(sv.y);
    // s_hat - y: -(v / cb + z) when v = cb (y - z - s_hat); s_hat - v / cb - z when v = cb (y - z)
    double rr = double(vv.x) / cb + double(zv.x), ri = double(vv.y) / cb + double(zv.y);
    if (!sub_s) {
      rr -= sr;
      ri -= si;
    }
    a += rr * rr + ri * ri;
    b += sr * sr + si * si;
  }
  const double ra = block_sum(a, sh);
  const double rb = block_sum(b, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ra;
    part[2 * blockIdx.x + 1] = rb;
  }
}

// weighted soft threshold + dual; grid (cdiv(per, 256), P), segment p thresholds at gamma_d[p]
__global__ __launch_bounds__(256) void prox_l1_kernel(int64_t per, const float* __restrict__ s, float* __restrict__ z,
                                                      const float* __restrict__ W, const float* __restrict__ gamma_d,
                                                      float gamma, float* __restrict__ v) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= per) return;
  const int64_t i = (int64_t)blockIdx.y * per + j;
  const float g = gamma_d ? gamma_d[blockIdx.y] : gamma;
  const float t = s[i] + z[i];
  const float tau = g * (W ? W[i] : 1.0f);
  const float m = fabsf(t) - tau;
  const float y = m > 0.f ? copysignf(m, t) : 0.f;
  const float zn = t - y;
  z[i] = zn;
  v[i] = y - zn;
}

// positive orthant + dual
__global__ __launch_bounds__(256) void prox_pos_kernel(int64_t N, const float* __restrict__ s, float* __restrict__ z,
                                                       float* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const float t = s[i] + z[i];
  const float y = fmaxf(t, 0.f);
  const float zn = t - y;
  z[i] = zn;
  v[i] = y - zn;
}

// per-chunk float64 partial sums of ||s + z - yhat||^2 and ||s - yhat||^2, s = cb s_in (cb: the block's
// weight, 1 without cblk)
__global__ __launch_bounds__(256) void ball_norms(const float2* __restrict__ s_in, const float2* __restrict__ z,
                                                  const float2* __restrict__ yh, const int4* __restrict__ chunks,
                                                  const float* __restrict__ cblk, double* __restrict__ part,
                                                  const int32_t* __restrict__ bmask) {
  __shared__ double sh[256];
  const int4 c = chunks[blockIdx.x];
  if (bmask && !bmask[c.x]) return;   // block not selected: its partials (and norms) are not used
  const float cb = cblk ? cblk[c.x] : 1.0f;
  double a = 0.0, b = 0.0;
  auto acc = [&](float2 si, float2 zv, float2 yv) {
    const float2 sv = make_float2(cb * si.x, cb * si.y);
    const double dr = double(sv.x) - double(yv.x), di = double(sv.y) - double(yv.y);
    const double tr = dr + double(zv.x), ti = di + double(zv.y);
    a += tr * tr + ti * ti;
    b += dr * dr + di * di;
  };
  int i = c.y + threadIdx.x;
  for (; i + 768 < c.z; i += 1024) {   // twelve loads in flight; the sums keep the order of i
    float2 sv[4], zv[4], yv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      sv[u] = s_in[i + 256 * u];
      zv[u] = z[i + 256 * u];
      yv[u] = yh[i + 256 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc(sv[u], zv[u], yv[u]);
  }
  for (; i < c.z; i += 256) acc(s_in[i], z[i], yh[i]);
  const double ra = block_sum(a, sh);
  const double rb = block_sum(b, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ra;
    part[2 * blockIdx.x + 1] = rb;
  }
}

// per block: rho = ||t - yhat||, resid = ||s - yhat|| (chunk partials summed in order); with bmask, blocks left
// out keep the values they hold (their partials were not computed)
__global__ void ball_final(const double* __restrict__ part, const int* __restrict__ first, int R,
                           double* __restrict__ rho, double* __restrict__ resid,
                           const int32_t* __restrict__ bmask) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= R || (bmask && !bmask[b])) return;
  double a = 0.0, c = 0.0;
  for (int k = first[b]; k < first[b + 1]; ++k) {
    a += part[2 * k];
    c += part[2 * k + 1];
  }
  rho[b] = sqrt(a);
  resid[b] = sqrt(c);
}

// s = cb s_in; y = yhat + (t - yhat) min(1, eps/rho); z <- t - y; v = cb (y - z (- s if sub_s)), the
// factor cb readying v for the unweighted adjoint
__global__ __launch_bounds__(256) void ball_project(const float2* __restrict__ s_in, float2* __restrict__ z,
                                                    const float2* __restrict__ yh, const int4* __restrict__ chunks,
                                                    const double* __restrict__ eps, const double* __restrict__ rho,
                                                    const float* __restrict__ cblk, float2* __restrict__ v, int sub_s) {
  const int4 c = chunks[blockIdx.x];
  const double r = rho[c.x], e = eps[c.x];
  const float cb = cblk ? cblk[c.x] : 1.0f;
  const bool inside = r <= e;   // inside the ball (boundary included) the projection is the identity
  const float ratio = inside ? 1.0f : float(e / r);
  auto step = [&](int i, float2 si, float2 zv, float2 yv) {
    const float2 sv = make_float2(cb * si.x, cb * si.y);
    const float tr = sv.x + zv.x, ti = sv.y + zv.y;
    const float yr = inside ? tr : yv.x + (tr - yv.x) * ratio;
    const float yi = inside ? ti : yv.y + (ti - yv.y) * ratio;
    const float zr = tr - yr, zi = ti - yi;
    z[i] = make_float2(zr, zi);
    const float vr = sub_s ? yr - zr - sv.x : yr - zr, vi = sub_s ? yi - zi - sv.y : yi - zi;
    v[i] = make_float2(cb * vr, cb * vi);
  };
  int i = c.y + threadIdx.x;
  for (; i + 768 < c.z; i += 1024) {   // twelve loads in flight
    float2 sv[4], zv[4], yv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      sv[u] = s_in[i + 256 * u];
      zv[u] = z[i + 256 * u];
      yv[u] = yh[i + 256 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) step(i + 256 * u, sv[u], zv[u], yv[u]);
  }
  for (; i < c.z; i += 256) step(i, s_in[i], z[i], yh[i]);
}

// The ball step of the selected blocks of a block-subset iteration (blocks with bmask[b] = 0 are left as
// they are): s = cb s_in; y = yhat + (t - yhat) min(1, eps/rho) with t = s + z; z <- t - y;
// v = cb (y - z) (no -s: the x-update of these iterations takes Phi_hat^T Phi_hat x from its own product)
// and dv = v_new - v_old, the change the running image Phi_hat^T v needs.
__global__ __launch_bounds__(256) void ball_project_delta(const float2* __restrict__ s_in, float2* __restrict__ z,
                                                          const float2* __restrict__ yh, const int4* __restrict__ chunks,
                                                          const double* __restrict__ eps, const double* __restrict__ rho,
                                                          const float* __restrict__ cblk, const int32_t* __restrict__ bmask,
                                                          float2* __restrict__ v, float2* __restrict__ dv) {
  const int4 c = chunks[blockIdx.x];
  if (!bmask[c.x]) return;
  const double r = rho[c.x], e = eps[c.x];
  const float cb = cblk ? cblk[c.x] : 1.0f;
  const bool inside = r <= e;
  const float ratio = inside ? 1.0f : float(e / r);
  for (int i = c.y + threadIdx.x; i < c.z; i += 256) {
    const float2 si = s_in[i], zv = z[i], yv = yh[i], vo = v[i];
    const float tr = cb * si.x + zv.x, ti = cb * si.y + zv.y;
    const float yr = inside ? tr : yv.x + (tr - yv.x) * ratio;
    const float yi = inside ? ti : yv.y + (ti - yv.y) * ratio;
    const float zr = tr - yr, zi = ti - yi;
    z[i] = make_float2(zr, zi);
    const float vr = cb * (yr - zr), vi = cb * (yi - zi);
    v[i] = make_float2(vr, vi);
    dv[i] = make_float2(vr - vo.x, vi - vo.y);
  }
}

__global__ __launch_bounds__(256) void reweight_kernel(int64_t per, const float* __restrict__ c,
                                                       const double* __restrict__ delta_d, double delta,
                                                       float* __restrict__ W) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= per) return;
  const int64_t i = (int64_t)blockIdx.y * per + j;
  const double dl = delta_d ? delta_d[blockIdx.y] : delta;
  const double den = dl + fabs(double(c[i]));
  W[i] = den > 0 ? float(dl / den) : 1.f;   // delta = 0 at a zero coefficient: the rule's value at c = 0
}

}  // namespace

namespace sh {

sh_status Reducer::init(int segments) {
  P = segments;
  rb = RB / P > 1 ? RB / P : 1;   // about RB work-groups in all
  SH_TRY(part.alloc(2 * size_t(P) * rb));
  SH_TRY(part2.alloc(size_t(P) * rb));
  return SH_OK;
}

sh_status Reducer::cg_init(const float* a, const float* b, const float* c, const float* x, float* r, float* p,
                           float* xprev, int64_t per, double* rs_out, hipStream_t st, float xc) {
  hipLaunchKernelGGL(cg_init_rr, dim3(rb, P), dim3(256), 0, st, a, b, c, x, r, p, xprev, per, part.ptr, xc);
  hipLaunchKernelGGL(sum_final, dim3(P), dim3(256), 0, st, part.ptr, rb, rs_out);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status Reducer::cg_ap(const float* p, float* Ap, int64_t per, hipStream_t st, float pc) {
  hipLaunchKernelGGL(cg_ap_dot, dim3(rb, P), dim3(256), 0, st, p, Ap, per, part.ptr, pc);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status Reducer::cg_update(float* x, float* r, const float* p, const float* Ap, int64_t per, const double* rs,
                             double* pap_out, hipStream_t st) {
  hipLaunchKernelGGL(cg_update_rr, dim3(rb, P), dim3(256), 0, st, x, r, p, Ap, per, rs, part.ptr, pap_out,
                     part2.ptr);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status Reducer::cg_dir(const float* r, float* p, int64_t per, const double* rs, double* rs_out, hipStream_t st) {
  hipLaunchKernelGGL(cg_dir_rr, dim3(rb, P), dim3(256), 0, st, r, p, per, rs, part2.ptr, rs_out);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status Reducer::change(const float* x, const float* xprev, int64_t per, double* out2, hipStream_t st) {
  hipLaunchKernelGGL(change_dots, dim3(rb, P), dim3(256), 0, st, x, xprev, per, part.ptr);
  hipLaunchKernelGGL(sum_final, dim3(2 * P), dim3(256), 0, st, part.ptr, rb, out2);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status Reducer::dot(const float* a, const float* b, int64_t per, double* out, hipStream_t st) {
  hipLaunchKernelGGL(dot_partial, dim3(rb, P), dim3(256), 0, st, a, b, per, part.ptr);
  hipLaunchKernelGGL(sum_final, dim3(P), dim3(256), 0, st, part.ptr, rb, out);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status Reducer::std_dev(const float* a, int64_t per, double* sum_out, double* var_out, hipStream_t st) {
  hipLaunchKernelGGL(mean_partial, dim3(rb, P), dim3(256), 0, st, a, per, part.ptr);
  hipLaunchKernelGGL(sum_final, dim3(P), dim3(256), 0, st, part.ptr, rb, sum_out);
  hipLaunchKernelGGL(var_partial, dim3(rb, P), dim3(256), 0, st, a, per, sum_out, part.ptr);
  hipLaunchKernelGGL(sum_final, dim3(P), dim3(256), 0, st, part.ptr, rb, var_out);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status Reducer::maxabs(const float* a, int64_t per, double* out, hipStream_t st) {
  hipLaunchKernelGGL(maxabs_partial, dim3(rb, P), dim3(256), 0, st, a, per, part.ptr);
  hipLaunchKernelGGL(max_final, dim3(P), dim3(256), 0, st, part.ptr, rb, out);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status Reducer::comb3_sq(const float* a, const float* b, const float* c, float fb, float fc, int64_t per, double* out,
                            hipStream_t st) {
  hipLaunchKernelGGL(comb3_sq_partial, dim3(rb, P), dim3(256), 0, st, a, b, c, fb, fc, per, part.ptr);
  hipLaunchKernelGGL(sum_final, dim3(P), dim3(256), 0, st, part.ptr, rb, out);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status Reducer::l1w(const float* c, const float* W, int64_t per, double* out, hipStream_t st) {
  hipLaunchKernelGGL(l1w_partial, dim3(rb, P), dim3(256), 0, st, c, W, per, part.ptr);
  hipLaunchKernelGGL(sum_final, dim3(P), dim3(256), 0, st, part.ptr, rb, out);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status launch_prox_l1(int64_t per, int P, const float* s, float* z, const float* W, const float* gamma_d,
                         float gamma, float* v, hipStream_t st) {
  ProfScope ps("prox", st);
  hipLaunchKernelGGL(prox_l1_kernel, dim3((unsigned)cdiv(per, 256), P), dim3(256), 0, st, per, s, z, W, gamma_d,
                     gamma, v);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status launch_prox_pos(int64_t N, const float* s, float* z, float* v, hipStream_t st) {
  ProfScope ps("prox", st);
  hipLaunchKernelGGL(prox_pos_kernel, dim3((unsigned)cdiv(N, 256)), dim3(256), 0, st, N, s, z, v);
  SH_LAUNCHED();
  return SH_OK;
}

// The three ball kernels (norm partials, per-block norms, projection) with no timing events.
sh_status ball_kernels(sh_op op, const float2* s, float2* z, const float2* yhat, const double* eps, double* rho,
                              double* resid, float2* v, bool sub_s, const float* cblk, hipStream_t st) {
  const unsigned nc = (unsigned)op->n_chunks;
  hipLaunchKernelGGL(ball_norms, dim3(nc), dim3(256), 0, st, s, z, yhat, op->chunks.ptr, cblk, op->partials.ptr,
                     (const int32_t*)nullptr);
  hipLaunchKernelGGL(ball_final, dim3((unsigned)cdiv(op->R, 64)), dim3(64), 0, st, op->partials.ptr,
                     op->chunk_first_d.ptr, op->R, rho, resid, (const int32_t*)nullptr);
  hipLaunchKernelGGL(ball_project, dim3(nc), dim3(256), 0, st, s, z, yhat, op->chunks.ptr, eps, rho, cblk, v,
                     sub_s ? 1 : 0);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status ball_norms_only(sh_op op, const float2* s, const float2* z, const float2* yhat, const float* cblk, double* rho,
                          double* resid, hipStream_t st) {
  const unsigned nc = (unsigned)op->n_chunks;
  hipLaunchKernelGGL(ball_norms, dim3(nc), dim3(256), 0, st, s, z, yhat, op->chunks.ptr, cblk, op->partials.ptr,
                     (const int32_t*)nullptr);
  hipLaunchKernelGGL(ball_final, dim3((unsigned)cdiv(op->R, 64)), dim3(64), 0, st, op->partials.ptr,
                     op->chunk_first_d.ptr, op->R, rho, resid, (const int32_t*)nullptr);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status launch_prox_ball(sh_op op, const float2* s, float2* z, const float2* yhat, const double* eps, double* rho,
                           double* resid, float2* v, bool sub_s, const float* cblk, hipStream_t st) {
  ProfScope ps("prox", st);
  return ball_kernels(op, s, z, yhat, eps, rho, resid, v, sub_s, cblk, st);
}

sh_status launch_kkt_vis(sh_op op, const float2* s, const float2* z, const float2* v, const float* cblk, double* prim_b,
                         double* scale_b, hipStream_t st, bool sub_s) {
  const unsigned nc = (unsigned)op->n_chunks;
  hipLaunchKernelGGL(kkt_vis_partial, dim3(nc), dim3(256), 0, st, s, z, v, op->chunks.ptr, cblk, op->partials.ptr,
                     sub_s ? 1 : 0);
  hipLaunchKernelGGL(ball_final, dim3((unsigned)cdiv(op->R, 64)), dim3(64), 0, st, op->partials.ptr,
                     op->chunk_first_d.ptr, op->R, prim_b, scale_b, (const int32_t*)nullptr);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status launch_prox_ball_subset(sh_op op, const float2* s, float2* z, const float2* yhat, const double* eps,
                                 double* rho, double* resid, float2* v, float2* dv, const float* cblk,
                                 const int32_t* bmask, hipStream_t st) {
  ProfScope ps("prox", st);
  const unsigned nc = (unsigned)op->n_chunks;
  hipLaunchKernelGGL(ball_norms, dim3(nc), dim3(256), 0, st, s, z, yhat, op->chunks.ptr, cblk, op->partials.ptr, bmask);
  hipLaunchKernelGGL(ball_final, dim3((unsigned)cdiv(op->R, 64)), dim3(64), 0, st, op->partials.ptr,
                     op->chunk_first_d.ptr, op->R, rho, resid, bmask);
  hipLaunchKernelGGL(ball_project_delta, dim3(nc), dim3(256), 0, st, s, z, yhat, op->chunks.ptr, eps, rho, cblk, bmask,
                     v, dv);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status launch_reweight(int64_t per, int P, const float* c, const double* delta_d, double delta, float* W,
                          hipStream_t st) {
  hipLaunchKernelGGL(reweight_kernel, dim3((unsigned)cdiv(per, 256), P), dim3(256), 0, st, per, c, delta_d, delta, W);
  SH_LAUNCHED();
  return SH_OK;
}

}  // namespace sh

// Per-block float64 norms of sh_prox_ball_noalloc: a file-scope device array (each GPU the library runs
// on holds its own copy until the process ends).  Host code never passes `scratch` itself: its address on
// each device comes from hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) double scratch[SH_BALL_NOALLOC_MAX_BLOCKS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of `scratch`, resolved on the first call on that device.
sh_status scratch_address(double** out) {
  int dev = -1;
  SH_HIP(hipGetDevice(&dev));
  SH_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index %d outside [0, %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    SH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    SH_REQUIRE(p != nullptr, "no device address for the ball-projection scratch on device %d", dev);
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return SH_OK;
}
}  // namespace

extern "C" {

sh_status sh_prox_l1(int64_t D, const float* s, float* z, const float* W, float gamma, float* v_out, void* stream) {
  SH_REQUIRE(D >= 1 && s && z && v_out, "invalid argument");
  SH_REQUIRE(std::isfinite(gamma) && gamma >= 0.f, "gamma must be finite and >= 0");
  return sh::launch_prox_l1(D, 1, s, z, W, nullptr, gamma, v_out, (hipStream_t)stream);
}

sh_status sh_prox_pos(int64_t N, const float* s, float* z, float* v_out, void* stream) {
  SH_REQUIRE(N >= 1 && s && z && v_out, "invalid argument");
  return sh::launch_prox_pos(N, s, z, v_out, (hipStream_t)stream);
}

sh_status sh_prox_ball(sh_op op, const float* s, float* z, const float* yhat, const double* eps, float* v_out,
                       double* resid_out, void* stream) {
  SH_REQUIRE(op && s && z && yhat && eps && v_out && resid_out, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  sh::DevBuf<double> rho;
  SH_TRY(rho.alloc(op->R));
  SH_TRY(sh::launch_prox_ball(op, (const float2*)s, (float2*)z, (const float2*)yhat, eps, rho.ptr, resid_out,
                              (float2*)v_out, false, nullptr, st));
  SH_HIP(hipStreamSynchronize(st));  // rho is freed on return
  return SH_OK;
}

sh_status sh_prox_ball_noalloc(sh_op op, const float* s, float* z, const float* yhat, const double* eps, float* v_out,
                               double* resid_out, void* stream) {
  SH_REQUIRE(op && s && z && yhat && eps && v_out && resid_out, "NULL argument");
  SH_REQUIRE(op->R <= SH_BALL_NOALLOC_MAX_BLOCKS, "%d blocks exceed the %d that sh_prox_ball_noalloc holds (use "
             "sh_prox_ball)", op->R, SH_BALL_NOALLOC_MAX_BLOCKS);
  double* rho = nullptr;
  SH_TRY(scratch_address(&rho));
  // ball_final writes every block's norm before ball_project reads it: nothing needs clearing
  return sh::ball_kernels(op, (const float2*)s, (float2*)z, (const float2*)yhat, eps, rho, resid_out, (float2*)v_out,
                          false, nullptr, (hipStream_t)stream);
}

sh_status sh_reweight(int64_t D, const float* c, double delta, float* W_out, void* stream) {
  SH_REQUIRE(D >= 1 && c && W_out, "invalid argument");
  SH_REQUIRE(std::isfinite(delta) && delta > 0, "delta must be finite and > 0");
  return sh::launch_reweight(D, 1, c, nullptr, delta, W_out, (hipStream_t)stream);
}

sh_status sh_std(int64_t D, const float* c, double* std_out, void* stream) {
  SH_REQUIRE(D >= 1 && c && std_out, "invalid argument");
  hipStream_t st = (hipStream_t)stream;
  sh::Reducer red;
  SH_TRY(red.init());
  sh::DevBuf<double> r;
  SH_TRY(r.alloc(2));
  SH_TRY(red.std_dev(c, D, r.ptr, r.ptr + 1, st));
  double h[2];
  SH_HIP(hipMemcpyAsync(h, r.ptr, sizeof(h), hipMemcpyDeviceToHost, st));
  SH_HIP(hipStreamSynchronize(st));
  *std_out = std::sqrt(h[1] / double(D));
  return SH_OK;
}

}  // extern "C"
