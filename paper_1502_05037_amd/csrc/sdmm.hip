// SDMM solve of the blocked problem (3) with SARA reweighting (PURIFY paragraph; SARA paragraph).
//
// The problem is min ||W Psi^dagger x||_1 over x >= 0 subject to ||y_i - Phi_i x|| <= eps_i, written
// as f_0(Psi^dagger x) + sum_i iota_{B_i}(Phi_i x) + iota_+(x).  SDMM keeps (y_j, z_j) per term:
//   x   = Q^{-1} sum_j L_j^T (y_j - z_j),  Q = Psi Psi^dagger + Phi^dagger Phi + I = 2I + Re(Phi^H Phi)
//   s_j = L_j x;  y_j = prox(s_j + z_j);  z_j += s_j - y_j.
// Everything runs on Phi_hat = Phi / nu (nu = ||Phi||), y_hat = y / nu, eps_hat = eps / nu, which
// keeps the solution set and puts the spectrum of Q in [2, 3].
//
// GPU layout: the state lives in device memory; visibility-space vectors are in internal order
// (blocks contiguous).  v_j = y_j - z_j is kept instead of y_j.  The x-update is conjugate gradients
// warm-started at x_{n-1} with a fixed number of steps; its initial residual
//   b - Q x_{n-1} = Psi v_psi + Phi_hat^dagger (v_phi - Phi_hat x_{n-1}) + v_+ - 2 x_{n-1}
// reuses s_phi = Phi_hat x_{n-1} from the previous iteration, so one iteration costs
// (cg_iters + 1) applications each of Phi and Phi^dagger.  CG scalars stay on the device.
// Block norms, dot products, the stopping test and the reweighting statistics are float64.
#include <chrono>
#include <cmath>
#include <memory>

#include "prox.hpp"

// Psi (dwt.hip)
extern "C" sh_status sh_psi_fwd(sh_psi psi, const float* coeffs, float* x, void* stream);
extern "C" sh_status sh_psi_adj(sh_psi psi, const float* x, float* coeffs, void* stream);
extern "C" sh_status sh_psi_planes(sh_psi psi, int32_t* q_out);
int psi_side(sh_psi psi);

namespace {

__global__ void fill_kernel(float* a, int64_t N, float v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) a[i] = v;
}

__global__ void scale_kernel(const float* __restrict__ a, float* __restrict__ b, int64_t N, const double* __restrict__ nrm2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double n2 = nrm2[0];
  const float s = n2 > 0 ? float(1.0 / sqrt(n2)) : 0.f;
  if (i < N) b[i] = a[i] * s;
}

__global__ void gather_scale(const float2* __restrict__ src, const uint32_t* __restrict__ idx, float2* __restrict__ dst,
                             int64_t M, float s) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < M) {
    const float2 v = src[idx[i]];
    dst[i] = make_float2(v.x * s, v.y * s);
  }
}

// r = a + b + c - 2x; p = r; xprev = x
__global__ void cg_init(const float* __restrict__ a, const float* __restrict__ b, const float* __restrict__ c,
                        const float* __restrict__ x, float* __restrict__ r, float* __restrict__ p,
                        float* __restrict__ xprev, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const float xv = x[i];
  const float rv = a[i] + b[i] + c[i] - 2.f * xv;
  r[i] = rv;
  p[i] = rv;
  xprev[i] = xv;
}

// Ap = 2p + Ap
__global__ void cg_ap(const float* __restrict__ p, float* __restrict__ Ap, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) Ap[i] = 2.f * p[i] + Ap[i];
}

// alpha = rs / pAp; x += alpha p; r -= alpha Ap
__global__ void cg_update(float* __restrict__ x, float* __restrict__ r, const float* __restrict__ p,
                          const float* __restrict__ Ap, int64_t N, const double* __restrict__ rs,
                          const double* __restrict__ pAp) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double d = pAp[0];
  const float alpha = d > 0 ? float(rs[0] / d) : 0.f;
  if (i < N) {
    x[i] = fmaf(alpha, p[i], x[i]);
    r[i] = fmaf(-alpha, Ap[i], r[i]);
  }
}

// beta = rs_new / rs; p = r + beta p
__global__ void cg_dir(const float* __restrict__ r, float* __restrict__ p, int64_t N, const double* __restrict__ rs,
                       const double* __restrict__ rs_new) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double d = rs[0];
  const float beta = d > 0 ? float(rs_new[0] / d) : 0.f;
  if (i < N) p[i] = fmaf(beta, p[i], r[i]);
}

__global__ void diff_kernel(const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ c, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) c[i] = a[i] - b[i];
}

inline unsigned nblk(int64_t n) { return (unsigned)sh::cdiv(n, 256); }

struct Work {
  sh::DevBuf<float> x, xprev, r, p, Ap, t1, t2, vpos, zpos;
  sh::DevBuf<float> spsi, zpsi, vpsi, W;
  sh::DevBuf<float2> yhat, sphi, zphi, vphi, vtmp;
  sh::DevBuf<double> sc, eps_hat, rho, resid;
  sh::Reducer red;
};

// Power iteration on Re(Phi^H Phi) (scale 1) from x0; returns sqrt of the Rayleigh quotient.
sh_status power_norm(sh_op op, const float* x0, int iters, double tol, double* nu, hipStream_t st) {
  const int64_t N = int64_t(op->n) * op->n;
  sh::DevBuf<float> x, y;
  sh::DevBuf<float2> v;
  sh::DevBuf<double> sc;
  sh::Reducer red;
  SH_TRY(x.alloc(N));
  SH_TRY(y.alloc(N));
  SH_TRY(v.alloc(op->M));
  SH_TRY(sc.alloc(4));
  SH_TRY(red.init());
  SH_TRY(red.dot(x0, x0, N, sc.ptr, st));
  hipLaunchKernelGGL(scale_kernel, dim3(nblk(N)), dim3(256), 0, st, x0, x.ptr, N, sc.ptr);
  double lam = 0.0;
  for (int it = 0; it < iters; ++it) {
    SH_TRY(sh::phi_forward(op, x.ptr, v.ptr, false, 1.f, st));
    SH_TRY(sh::phi_adjoint(op, v.ptr, y.ptr, false, 1.f, st));
    SH_TRY(red.dot(x.ptr, y.ptr, N, sc.ptr + 1, st));
    SH_TRY(red.dot(y.ptr, y.ptr, N, sc.ptr + 2, st));
    hipLaunchKernelGGL(scale_kernel, dim3(nblk(N)), dim3(256), 0, st, y.ptr, x.ptr, N, sc.ptr + 2);
    double h[2];
    SH_HIP(hipMemcpyAsync(h, sc.ptr + 1, sizeof(h), hipMemcpyDeviceToHost, st));
    SH_HIP(hipStreamSynchronize(st));
    if (!std::isfinite(h[0]) || !std::isfinite(h[1])) {
      sh::set_error("non-finite value in power iteration");
      return SH_ENONFINITE;
    }
    const double lam_new = h[0];
    const bool done = lam > 0 && std::fabs(lam_new - lam) <= tol * lam_new;
    lam = lam_new;
    if (done) break;
  }
  *nu = std::sqrt(std::max(lam, 0.0));
  return SH_OK;
}

}  // namespace

extern "C" {

void sh_sdmm_default_params(sh_sdmm_params* p) {
  if (!p) return;
  p->gamma = -1.0;
  p->nu = -1.0;
  p->tol_rel = 0.0;
  p->eps_slack = 1e-4;
  p->rw_beta = 0.5;
  p->rw_delta0 = 0.0;
  p->max_iter = 300;
  p->cg_iters = 8;
  p->passes = 1;
  p->check_every = 10;
}

sh_status sh_op_norm(sh_op op, const float* x0, int32_t iters, double tol, double* nu_out, void* stream) {
  SH_REQUIRE(op && x0 && nu_out, "NULL argument");
  SH_REQUIRE(iters >= 1 && tol >= 0, "iters >= 1 and tol >= 0 required");
  return power_norm(op, x0, iters, tol, nu_out, (hipStream_t)stream);
}

}  // extern "C"

struct sh_sdmm_s {
  sh_op op = nullptr;
  sh_psi psi = nullptr;
  sh_sdmm_params prm{};
  Work w;
  int64_t N = 0, M = 0, D = 0;
  int R = 0, kcg = 0;
  double nu = 0, gamma = 0, delta = 0;
  float inv_nu = 1.f;
  std::vector<double> eh;          // eps / nu (host)
  const float* Wp = nullptr;       // weights of the current pass (NULL = identity)
  int iters_total = 0;
  double *s_rs = nullptr, *s_pap = nullptr, *s_misc = nullptr;
};

namespace {

sh_status sdmm_setup(sh_sdmm s, const float* y, const double* eps, const float* W0, const float* x0, hipStream_t st) {
  sh_op op = s->op;
  const int R = s->R;
  const int64_t N = s->N, M = s->M, D = s->D;
  const int kcg = s->kcg;
  Work& w = s->w;
  for (auto* b : {&w.x, &w.xprev, &w.r, &w.p, &w.Ap, &w.t1, &w.t2, &w.vpos, &w.zpos}) SH_TRY(b->alloc(N));
  for (auto* b : {&w.spsi, &w.zpsi, &w.vpsi, &w.W}) SH_TRY(b->alloc(D));
  for (auto* b : {&w.yhat, &w.sphi, &w.zphi, &w.vphi, &w.vtmp}) SH_TRY(b->alloc(M));
  SH_TRY(w.sc.alloc(2 * kcg + 16));
  SH_TRY(w.eps_hat.alloc(R));
  SH_TRY(w.rho.alloc(R));
  SH_TRY(w.resid.alloc(R));
  SH_TRY(w.red.init());
  double* sc = w.sc.ptr;
  s->s_rs = sc;                  // rs_k, k = 0..kcg
  s->s_pap = sc + kcg + 1;       // pAp_k, k = 0..kcg-1
  s->s_misc = sc + 2 * kcg + 2;  // [0] dx^2, [1] x^2, [2] scratch, [3] objective, [4] scratch
  double* s_misc = s->s_misc;
  SH_HIP(hipMemsetAsync(w.resid.ptr, 0, R * sizeof(double), st));
  SH_HIP(hipMemsetAsync(w.sc.ptr, 0, (2 * kcg + 16) * sizeof(double), st));

  // non-finite data check (float64 sum of squares)
  SH_TRY(w.red.dot(y, y, 2 * M, s_misc + 2, st));
  double ysq = 0;
  SH_HIP(hipMemcpyAsync(&ysq, s_misc + 2, sizeof(double), hipMemcpyDeviceToHost, st));
  SH_HIP(hipStreamSynchronize(st));
  if (!std::isfinite(ysq)) {
    sh::set_error("visibilities contain non-finite values");
    return SH_ENONFINITE;
  }
  // normalisation nu
  double nu = s->prm.nu;
  if (!(nu > 0)) {
    hipLaunchKernelGGL(fill_kernel, dim3(nblk(N)), dim3(256), 0, st, w.t1.ptr, N, 1.f);
    SH_TRY(power_norm(op, w.t1.ptr, 200, 1e-12, &nu, st));
  }
  SH_REQUIRE(nu > 0 && std::isfinite(nu), "operator norm must be positive");
  s->nu = nu;
  s->inv_nu = float(1.0 / nu);
  hipLaunchKernelGGL(gather_scale, dim3(nblk(M)), dim3(256), 0, st, (const float2*)y, op->perm.ptr, w.yhat.ptr, M,
                     s->inv_nu);
  s->eh.resize(R);
  for (int i = 0; i < R; ++i) s->eh[i] = eps[i] / nu;
  SH_HIP(hipMemcpyAsync(w.eps_hat.ptr, s->eh.data(), R * sizeof(double), hipMemcpyHostToDevice, st));
  // gamma = 1e-3 max |Psi^dagger Phi^dagger y| / nu^2 unless given
  double gamma = s->prm.gamma;
  if (!(gamma > 0)) {
    SH_TRY(sh::phi_adjoint(op, (const float2*)y, w.t1.ptr, true, 1.f, st));
    SH_TRY(sh_psi_adj(s->psi, w.t1.ptr, w.spsi.ptr, st));
    SH_TRY(w.red.maxabs(w.spsi.ptr, D, s_misc + 2, st));
    double mx = 0;
    SH_HIP(hipMemcpyAsync(&mx, s_misc + 2, sizeof(double), hipMemcpyDeviceToHost, st));
    SH_HIP(hipStreamSynchronize(st));
    gamma = 1e-3 * mx / (nu * nu);
  }
  SH_REQUIRE(gamma > 0 && std::isfinite(gamma), "gamma must be positive (is y zero?)");
  s->gamma = gamma;
  // weights of the first pass
  if (W0) {
    SH_HIP(hipMemcpyAsync(w.W.ptr, W0, D * sizeof(float), hipMemcpyDeviceToDevice, st));
    s->Wp = w.W.ptr;
  }
  s->delta = s->prm.rw_delta0 > 0 && W0 ? s->prm.rw_delta0 : 0.0;
  // initial state: zero, or y_psi = Psi^dagger x0, y_phi = Phi_hat x0, y_+ = x0, z = 0
  SH_HIP(hipMemsetAsync(w.zpsi.ptr, 0, D * sizeof(float), st));
  SH_HIP(hipMemsetAsync(w.zphi.ptr, 0, M * sizeof(float2), st));
  SH_HIP(hipMemsetAsync(w.zpos.ptr, 0, N * sizeof(float), st));
  SH_HIP(hipMemsetAsync(w.vphi.ptr, 0, M * sizeof(float2), st));  // y_phi - z_phi - Phi_hat x0 = 0 either way
  if (x0) {
    SH_HIP(hipMemcpyAsync(w.x.ptr, x0, N * sizeof(float), hipMemcpyDeviceToDevice, st));
    SH_HIP(hipMemcpyAsync(w.vpos.ptr, x0, N * sizeof(float), hipMemcpyDeviceToDevice, st));
    SH_TRY(sh_psi_adj(s->psi, x0, w.vpsi.ptr, st));
    SH_TRY(sh::phi_forward(op, x0, w.sphi.ptr, false, s->inv_nu, st));
  } else {
    SH_HIP(hipMemsetAsync(w.x.ptr, 0, N * sizeof(float), st));
    SH_HIP(hipMemsetAsync(w.vpos.ptr, 0, N * sizeof(float), st));
    SH_HIP(hipMemsetAsync(w.vpsi.ptr, 0, D * sizeof(float), st));
    SH_HIP(hipMemsetAsync(w.sphi.ptr, 0, M * sizeof(float2), st));
  }
  SH_HIP(hipMemsetAsync(w.xprev.ptr, 0, N * sizeof(float), st));
  return SH_OK;
}

// One SDMM iteration, enqueued on `st` with no host synchronisation.
sh_status sdmm_step(sh_sdmm s, hipStream_t st) {
  sh_op op = s->op;
  Work& w = s->w;
  const int64_t N = s->N, D = s->D;
  const unsigned gN = nblk(N);
  const float inv_nu = s->inv_nu;
  double *s_rs = s->s_rs, *s_pap = s->s_pap, *s_misc = s->s_misc;
  // ---- x-update by CG from x_{n-1}
  SH_TRY(sh_psi_fwd(s->psi, w.vpsi.ptr, w.t1.ptr, st));
  SH_TRY(sh::phi_adjoint(op, w.vphi.ptr, w.t2.ptr, false, inv_nu, st));
  hipLaunchKernelGGL(cg_init, dim3(gN), dim3(256), 0, st, w.t1.ptr, w.t2.ptr, w.vpos.ptr, w.x.ptr, w.r.ptr, w.p.ptr,
                     w.xprev.ptr, N);
  SH_TRY(w.red.dot(w.r.ptr, w.r.ptr, N, s_rs, st));
  for (int k = 0; k < s->kcg; ++k) {
    SH_TRY(sh::phi_forward(op, w.p.ptr, w.vtmp.ptr, false, inv_nu, st));
    SH_TRY(sh::phi_adjoint(op, w.vtmp.ptr, w.Ap.ptr, false, inv_nu, st));
    hipLaunchKernelGGL(cg_ap, dim3(gN), dim3(256), 0, st, w.p.ptr, w.Ap.ptr, N);
    SH_TRY(w.red.dot(w.p.ptr, w.Ap.ptr, N, s_pap + k, st));
    hipLaunchKernelGGL(cg_update, dim3(gN), dim3(256), 0, st, w.x.ptr, w.r.ptr, w.p.ptr, w.Ap.ptr, N, s_rs + k,
                       s_pap + k);
    if (k + 1 < s->kcg) {
      SH_TRY(w.red.dot(w.r.ptr, w.r.ptr, N, s_rs + k + 1, st));
      hipLaunchKernelGGL(cg_dir, dim3(gN), dim3(256), 0, st, w.r.ptr, w.p.ptr, N, s_rs + k, s_rs + k + 1);
    }
  }
  SH_LAUNCHED();
  // ---- relative change
  hipLaunchKernelGGL(diff_kernel, dim3(gN), dim3(256), 0, st, w.x.ptr, w.xprev.ptr, w.t1.ptr, N);
  SH_TRY(w.red.dot(w.t1.ptr, w.t1.ptr, N, s_misc, st));
  SH_TRY(w.red.dot(w.x.ptr, w.x.ptr, N, s_misc + 1, st));
  // ---- splits
  SH_TRY(sh_psi_adj(s->psi, w.x.ptr, w.spsi.ptr, st));
  SH_TRY(sh::launch_prox_l1(D, w.spsi.ptr, w.zpsi.ptr, s->Wp, float(s->gamma), w.vpsi.ptr, st));
  SH_TRY(sh::phi_forward(op, w.x.ptr, w.sphi.ptr, false, inv_nu, st));
  SH_TRY(sh::launch_prox_ball(op, w.sphi.ptr, w.zphi.ptr, w.yhat.ptr, w.eps_hat.ptr, w.rho.ptr, w.resid.ptr,
                              w.vphi.ptr, true, st));
  SH_TRY(sh::launch_prox_pos(N, w.x.ptr, w.zpos.ptr, w.vpos.ptr, st));
  s->iters_total += 1;
  return SH_OK;
}

// Reads the stopping quantities of the last iteration (synchronises): rel change, residuals (hat units).
sh_status sdmm_read(sh_sdmm s, double* rel, std::vector<double>& hres, hipStream_t st) {
  double h[2];
  SH_HIP(hipMemcpyAsync(h, s->s_misc, sizeof(h), hipMemcpyDeviceToHost, st));
  hres.resize(s->R);
  SH_HIP(hipMemcpyAsync(hres.data(), s->w.resid.ptr, s->R * sizeof(double), hipMemcpyDeviceToHost, st));
  SH_HIP(hipStreamSynchronize(st));
  if (!std::isfinite(h[0]) || !std::isfinite(h[1])) {
    sh::set_error("non-finite iterate after %d iterations", s->iters_total);
    return SH_ENONFINITE;
  }
  *rel = h[1] > 0 ? std::sqrt(h[0] / h[1]) : (h[0] == 0 ? 0.0 : INFINITY);
  return SH_OK;
}

// Reweighting after a pass: delta_1 = std(Psi^dagger x) (float64), then delta <- beta delta.
sh_status sdmm_reweight(sh_sdmm s, float* W_dst, hipStream_t st) {
  Work& w = s->w;
  if (!(s->delta > 0)) {
    // sum of the coefficients in s_misc[2], sum of squared deviations in s_misc[4]
    SH_TRY(w.red.std_dev(w.spsi.ptr, s->D, s->s_misc + 2, s->s_misc + 4, st));
    double var_sum = 0;
    SH_HIP(hipMemcpyAsync(&var_sum, s->s_misc + 4, sizeof(double), hipMemcpyDeviceToHost, st));
    SH_HIP(hipStreamSynchronize(st));
    s->delta = std::sqrt(var_sum / double(s->D));
  } else {
    s->delta *= s->prm.rw_beta;
  }
  if (!(s->delta > 0) || !std::isfinite(s->delta)) {
    sh::set_error("reweighting delta is %g (zero image?)", s->delta);
    return s->delta == 0 ? SH_EINVAL : SH_ENONFINITE;
  }
  return sh::launch_reweight(s->D, w.spsi.ptr, s->delta, W_dst, st);
}

sh_status sdmm_validate(sh_op op, sh_psi psi, const float* y, const double* eps, const sh_sdmm_params* prm) {
  SH_REQUIRE(op && psi && y && eps && prm, "NULL argument");
  SH_REQUIRE(psi_side(psi) == op->n, "psi and op image sides differ");
  SH_REQUIRE(prm->max_iter >= 1 && prm->cg_iters >= 1 && prm->cg_iters <= 64 && prm->passes >= 1 &&
                 prm->check_every >= 1,
             "max_iter, passes, check_every >= 1 and cg_iters in [1, 64] required");
  SH_REQUIRE(prm->tol_rel >= 0 && prm->eps_slack >= 0 && prm->rw_beta > 0 && std::isfinite(prm->rw_beta),
             "tol_rel, eps_slack >= 0 and rw_beta > 0 required");
  for (int i = 0; i < op->R; ++i) {
    if (!std::isfinite(eps[i])) {
      sh::set_error("eps[%d] is not finite", i);
      return SH_ENONFINITE;
    }
    SH_REQUIRE(eps[i] > 0, "eps[%d] = %g must be > 0", i, eps[i]);
  }
  return SH_OK;
}

}  // namespace

extern "C" {

sh_status sh_sdmm_create(sh_op op, sh_psi psi, const float* y, const double* eps, const float* W, const float* x0,
                         const sh_sdmm_params* params, sh_sdmm* out, void* stream) {
  SH_REQUIRE(out, "out is NULL");
  *out = nullptr;
  SH_TRY(sdmm_validate(op, psi, y, eps, params));
  sh_sdmm s = new (std::nothrow) sh_sdmm_s();
  if (!s) {
    sh::set_error("host allocation failed");
    return SH_ENOMEM;
  }
  s->op = op;
  s->psi = psi;
  s->prm = *params;
  int32_t q = 0;
  sh_psi_planes(psi, &q);
  s->N = int64_t(op->n) * op->n;
  s->M = op->M;
  s->D = int64_t(q) * s->N;
  s->R = op->R;
  s->kcg = params->cg_iters;
  sh_status st = sdmm_setup(s, y, eps, W, x0, (hipStream_t)stream);
  if (st == SH_OK) st = hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? SH_OK : SH_EDEVICE;
  if (st != SH_OK) {
    delete s;
    return st;
  }
  *out = s;
  return SH_OK;
}

sh_status sh_sdmm_iterate(sh_sdmm s, int32_t iters, void* stream) {
  SH_REQUIRE(s && iters >= 0, "invalid argument");
  for (int i = 0; i < iters; ++i) SH_TRY(sdmm_step(s, (hipStream_t)stream));
  return SH_OK;
}

sh_status sh_sdmm_result(sh_sdmm s, float* x_out, double* block_resid, double* rel_change, void* stream) {
  SH_REQUIRE(s, "NULL session");
  hipStream_t st = (hipStream_t)stream;
  if (x_out) SH_HIP(hipMemcpyAsync(x_out, s->w.x.ptr, s->N * sizeof(float), hipMemcpyDeviceToDevice, st));
  double rel = 0;
  std::vector<double> hres;
  SH_TRY(sdmm_read(s, &rel, hres, st));
  if (block_resid)
    for (int i = 0; i < s->R; ++i) block_resid[i] = hres[i] * s->nu;
  if (rel_change) *rel_change = rel;
  return SH_OK;
}

sh_status sh_sdmm_destroy(sh_sdmm s) {
  delete s;
  return SH_OK;
}

sh_status sh_sdmm_solve(sh_op op, sh_psi psi, const float* y, const double* eps, const float* W0, const float* x0,
                        const sh_sdmm_params* prm, float* x_out, float* W_out, double* block_resid,
                        sh_sdmm_info* info, void* stream) {
  const auto t_start = std::chrono::steady_clock::now();
  SH_REQUIRE(x_out, "x_out is NULL");
  sh_sdmm s = nullptr;
  SH_TRY(sh_sdmm_create(op, psi, y, eps, W0, x0, prm, &s, stream));
  std::unique_ptr<sh_sdmm_s> guard(s);
  hipStream_t st = (hipStream_t)stream;
  sh_sdmm_info inf{};
  inf.gamma = s->gamma;
  inf.nu = s->nu;
  std::vector<double> hres;
  double rel = INFINITY;
  bool converged = false;
  int it_last = 0;
  for (int pass = 0; pass < prm->passes; ++pass) {
    converged = false;
    int it = 0;
    while (it < prm->max_iter) {
      SH_TRY(sdmm_step(s, st));
      ++it;
      if (prm->tol_rel > 0 && (it % prm->check_every == 0 || it == prm->max_iter)) {
        SH_TRY(sdmm_read(s, &rel, hres, st));
        bool feas = true;
        for (int i = 0; i < s->R; ++i) feas = feas && hres[i] <= s->eh[i] * (1.0 + prm->eps_slack);
        if (rel <= prm->tol_rel && feas) {
          converged = true;
          break;
        }
      }
    }
    it_last = it;
    inf.iters_total += it;
    inf.passes_done = pass + 1;
    // objective with this pass's weights; spsi holds Psi^dagger x_n
    if (pass + 1 == prm->passes) SH_TRY(s->w.red.l1w(s->w.spsi.ptr, s->Wp, s->D, s->s_misc + 3, st));
    // reweight for the next pass (or for W_out after the last one)
    if (pass + 1 < prm->passes) {
      SH_TRY(sdmm_reweight(s, s->w.W.ptr, st));
      s->Wp = s->w.W.ptr;
    } else if (W_out) {
      SH_TRY(sdmm_reweight(s, W_out, st));
    }
  }
  double obj = 0;
  SH_HIP(hipMemcpyAsync(&obj, s->s_misc + 3, sizeof(double), hipMemcpyDeviceToHost, st));
  SH_TRY(sh_sdmm_result(s, x_out, block_resid, &rel, stream));
  inf.converged = converged ? 1 : 0;
  inf.iters_last = it_last;
  inf.rel_change = rel;
  inf.objective = obj;
  inf.delta = s->delta;
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (info) *info = inf;
  return SH_OK;
}

}  // extern "C"
