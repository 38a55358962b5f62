// SDMM solve of the blocked problem (3) with SARA reweighting (PURIFY paragraph; SARA paragraph).
//
// The problem is min ||W Psi^dagger x||_1 over x >= 0 subject to ||y_i - Phi_i x|| <= eps_i, written
// as f_0(Psi^dagger x) + sum_i iota_{B_i}(Phi_i x) + iota_+(x).  SDMM keeps (y_j, z_j) per term:
//   x   = Q^{-1} sum_j L_j^T (y_j - z_j),  Q = Psi Psi^dagger + Phi^dagger Phi + I = 2I + Re(Phi^H Phi)
//   s_j = L_j x;  y_j = prox(s_j + z_j);  z_j += s_j - y_j.
// Everything runs on the normalised splits Phi_hat_b = c_b Phi_b, y_hat_b = c_b y_b, eps_hat_b = c_b eps_b
// with c_b = a_b / nu_p for block b of problem p: a_b = 1 (one normalisation per problem) or the
// density estimate of 1 / ||Phi_b|| (option block_norm, blocknorm.hip), and nu_p the norm of the
// a-weighted operator of problem p.  Any c_b > 0 keeps the solution set; this choice puts the
// spectrum of Q in [2, 3].
//
// GPU layout: the state lives in device memory; visibility-space vectors are in internal order
// (blocks contiguous).  v_j = y_j - z_j is kept instead of y_j.  The x-update is conjugate gradients
// warm-started at x_{n-1} with a fixed number of steps; its initial residual
//   b - Q x_{n-1} = Psi v_psi + Phi_hat^dagger (v_phi - Phi_hat x_{n-1}) + v_+ - 2 x_{n-1}
// reuses s_phi = Phi x_{n-1} from the previous iteration (stored unweighted; the ball step applies c_b,
// and v_phi leaves it multiplied by c_b for the adjoint).  The CG products Re(Phi_hat^H Phi_hat) p
// go through the Toeplitz embedding of that operator (toeplitz.hip: FFT passes only) or, with the
// option off, through a Phi, Phi^dagger pair; one iteration then costs one application each of Phi
// and Phi^dagger plus cg_iters Toeplitz products, or (cg_iters + 1) pairs.  CG scalars stay on the
// device.
// Block norms, dot products, the stopping test and the reweighting statistics are float64.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <cmath>
#include <memory>

#include "prox.hpp"

// Psi (dwt.hip)
extern "C" sh_status sh_psi_fwd(sh_psi psi, const float* coeffs, float* x, void* stream);
extern "C" sh_status sh_psi_adj(sh_psi psi, const float* x, float* coeffs, void* stream);
extern "C" sh_status sh_psi_planes(sh_psi psi, int32_t* q_out);
int psi_side(sh_psi psi);
int psi_batch(sh_psi psi);

namespace {

__global__ void fill_kernel(float* a, int64_t N, float v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) a[i] = v;
}

// Per-problem kernels run on grid (cdiv(per, 256), P): element j of segment p = blockIdx.y.
#define SEG_INDEX(per)                                      \
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; \
  if (j >= (per)) return;                                   \
  const int p = blockIdx.y;                                 \
  const int64_t i = (int64_t)p * (per) + j;

// b = a / sqrt(nrm2[p]) per segment
__global__ void scale_kernel(const float* __restrict__ a, float* __restrict__ b, int64_t per,
                             const double* __restrict__ nrm2) {
  SEG_INDEX(per)
  const double n2 = nrm2[p];
  const float sc = n2 > 0 ? float(1.0 / sqrt(n2)) : 0.f;
  b[i] = a[i] * sc;
}

// yhat (internal order) = c_b y[perm] for the block b of each chunk; one work-group per reduction chunk
__global__ __launch_bounds__(256) void gather_scale(const float2* __restrict__ src, const uint32_t* __restrict__ idx,
                                                    float2* __restrict__ dst, const int4* __restrict__ chunks,
                                                    const float* __restrict__ cblk) {
  const int4 c = chunks[blockIdx.x];
  const float s = cblk[c.x];
  for (int i = c.y + threadIdx.x; i < c.z; i += 256) {
    const float2 v = src[idx[i]];
    dst[i] = make_float2(v.x * s, v.y * s);
  }
}

// Dual warm start of the l1 split at s = Psi^dagger x0: the soft threshold's own split of s,
// y = soft(s, gamma_p W), z = s - y (= s clipped to [-gamma_p W, gamma_p W], the subgradient gamma W sign(s)
// where |s| exceeds the threshold); v = y - z.
__global__ void dual_l1_init(const float* __restrict__ sv, const float* __restrict__ W, const float* __restrict__ gamma,
                             float* __restrict__ z, float* __restrict__ v, int64_t per) {
  SEG_INDEX(per)
  const float c = sv[i];
  const float tau = gamma[p] * W[i];
  const float m = fabsf(c) - tau;
  const float y = m > 0.f ? copysignf(m, c) : 0.f;
  const float zz = c - y;
  z[i] = zz;
  v[i] = y - zz;
}
#undef SEG_INDEX

// Data splits at the warm start, per reduction chunk (one block each): s_hat = c_b s, y = the projection of
// s_hat onto block b's ball, z = lambda_p (y - yhat) (a multiple of the ball's outward normal at y, as at
// a fixed point), v = c_b (y - z - s_hat).  With mode 0 only u = c_b (y - yhat) is written (to v), the
// vector whose adjoint fixes lambda.
__global__ __launch_bounds__(256) void dual_ball_init(const float2* __restrict__ s_in, const float2* __restrict__ yh,
                                                      const int4* __restrict__ chunks, const float* __restrict__ cblk,
                                                      const double* __restrict__ eps, const double* __restrict__ rho,
                                                      const int* __restrict__ block_prob,
                                                      const double* __restrict__ lambda, float2* __restrict__ z,
                                                      float2* __restrict__ v, int mode) {
  const int4 c = chunks[blockIdx.x];
  const float cb = cblk[c.x];
  const double r = rho[c.x], e = eps[c.x];
  const float ratio = r <= e ? 1.0f : float(e / r);
  const float lam = mode ? float(lambda[block_prob[c.x]]) : 0.f;
  for (int i = c.y + threadIdx.x; i < c.z; i += 256) {
    const float2 si = s_in[i], yv = yh[i];
    const float sr = cb * si.x, sim = cb * si.y;
    const float dr = (sr - yv.x) * ratio, di = (sim - yv.y) * ratio;   // y - yhat
    if (!mode) {
      v[i] = make_float2(cb * dr, cb * di);
    } else {
      const float zr = lam * dr, zi = lam * di;
      z[i] = make_float2(zr, zi);
      v[i] = make_float2(cb * (yv.x + dr - zr - sr), cb * (yv.y + di - zi - sim));
    }
  }
}

// Block-subset iterations: block b takes part in iteration k when u(k R + b) < fraction, u(c) the c-th output
// (from 0) of the SplitMix64 sequence seeded with `seed` (Steele, Lea & Flood 2014), taken to [0, 1) by its top
// 53 bits.  One work-group; the iteration counter lives on the device and advances here, so that a captured
// iteration draws a new subset at every replay.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(1024) void block_mask_kernel(uint64_t seed, unsigned long long* __restrict__ ctr, int R,
                                                          double fraction, int32_t* __restrict__ mask) {
  const unsigned long long k = *ctr;
  for (int b = threadIdx.x; b < R; b += blockDim.x) {
    const uint64_t z = splitmix64_at(seed, (uint64_t)k * (uint64_t)R + (uint64_t)b);
    mask[b] = double(z >> 11) * 0x1.0p-53 < fraction ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) *ctr = k + 1;
}

// out = a + b - c (images)
__global__ void comb_kernel(float* __restrict__ out, const float* __restrict__ a, const float* __restrict__ b,
                            const float* __restrict__ c, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) out[i] = a[i] + b[i] - c[i];
}

__global__ void copy_kernel(float* __restrict__ dst, const float* __restrict__ src, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) dst[i] = src[i];
}

// c = a - b (images)
__global__ void sub_kernel(const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ c, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) c[i] = a[i] - b[i];
}

// a += b (images)
__global__ void add_kernel(float* __restrict__ a, const float* __restrict__ b, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) a[i] += b[i];
}

// v = c_b^2 s per chunk (the data splits' v = c_b (y - z) at a warm start y = c_b Phi x0, z = 0)
__global__ __launch_bounds__(256) void scale2_chunks(const float2* __restrict__ sv, float2* __restrict__ v,
                                                     const int4* __restrict__ chunks, const float* __restrict__ cblk) {
  const int4 c = chunks[blockIdx.x];
  const float q = cblk[c.x] * cblk[c.x];
  for (int i = c.y + threadIdx.x; i < c.z; i += 256) v[i] = make_float2(q * sv[i].x, q * sv[i].y);
}

inline unsigned nblk(int64_t n) { return (unsigned)sh::cdiv(n, 256); }

struct Work {
  sh::DevBuf<float> x, xprev, r, p, Ap, t1, t2, vpos, zpos;
  sh::DevBuf<float> spsi, zpsi, vpsi, W;
  sh::DevBuf<float2> yhat, sphi, zphi, vphi, vtmp;
  sh::DevBuf<double> sc, eps_hat, rho, resid, delta;
  sh::DevBuf<double> kkt;          // KKT reductions at exit: 8 per problem, then 2 per block
  sh::DevBuf<float> cblk, gamma;   // c_b per block, gamma per problem
  // block-subset iterations: the selected blocks, the iteration counter, the running image Phi_hat^T v_phi
  sh::DevBuf<int32_t> bmask;
  sh::DevBuf<unsigned long long> ctr;
  sh::DevBuf<float> bphi;
  // synthesis prior: the coefficients alpha (x = Psi alpha), the CG vectors in coefficient space, and the
  // coefficients taken with each problem's returned image
  sh::DevBuf<float> alpha, ar, ap, aAp, alpha_out;
  sh::Reducer red;
  sh_toep_s toep;                  // Re(Phi_hat^H Phi_hat) as a convolution (option toeplitz)
};

// Power iteration on Re(Phi^H Phi) (scale 1) from x0, for the P problems of the plan at once (each
// normalised and tested on its own); nu[p] = sqrt of problem p's Rayleigh quotient.  Stops when
// every problem's estimate changed by <= tol relative, or after `iters` steps.  With wblk (device,
// per block) the operator is sum_b wblk_b^2 Re(Phi_b^H Phi_b); with toep it is that Toeplitz operator.
sh_status power_norm(sh_op op, const float* x0, int iters, double tol, double* nu, hipStream_t st,
                     const float* wblk = nullptr, const sh_toep_s* toep = nullptr) {
  const int P = op->P;
  const int64_t per = int64_t(op->n) * op->n, N = per * P;
  sh::DevBuf<float> x, y;
  sh::DevBuf<float2> v;
  sh::DevBuf<double> sc;
  sh::Reducer red;
  SH_TRY(x.alloc(N));
  SH_TRY(y.alloc(N));
  SH_TRY(v.alloc(op->M));
  SH_TRY(sc.alloc(3 * P));
  SH_TRY(red.init(P));
  SH_TRY(red.dot(x0, x0, per, sc.ptr, st));
  hipLaunchKernelGGL(scale_kernel, dim3(nblk(per), P), dim3(256), 0, st, x0, x.ptr, per, sc.ptr);
  std::vector<double> lam(P, 0.0), h(2 * P);
  for (int it = 0; it < iters; ++it) {
    if (toep) {
      SH_TRY(sh::toeplitz_apply(op, toep->Ht.ptr, x.ptr, toep->tq.ptr, y.ptr, st));
    } else {
      SH_TRY(sh::phi_forward(op, x.ptr, v.ptr, false, wblk, st));
      SH_TRY(sh::phi_adjoint(op, v.ptr, y.ptr, false, wblk, st));
    }
    SH_TRY(red.dot(x.ptr, y.ptr, per, sc.ptr + P, st));
    SH_TRY(red.dot(y.ptr, y.ptr, per, sc.ptr + 2 * P, st));
    hipLaunchKernelGGL(scale_kernel, dim3(nblk(per), P), dim3(256), 0, st, y.ptr, x.ptr, per, sc.ptr + 2 * P);
    SH_HIP(hipMemcpyAsync(h.data(), sc.ptr + P, 2 * P * sizeof(double), hipMemcpyDeviceToHost, st));
    SH_HIP(hipStreamSynchronize(st));
    bool done = true;
    for (int p = 0; p < P; ++p) {
      if (!std::isfinite(h[p]) || !std::isfinite(h[P + p])) {
        sh::set_error("non-finite value in power iteration (problem %d)", p);
        return SH_ENONFINITE;
      }
      done = done && lam[p] > 0 && std::fabs(h[p] - lam[p]) <= tol * h[p];
      lam[p] = h[p];
    }
    if (done) break;
  }
  for (int p = 0; p < P; ++p) nu[p] = std::sqrt(std::max(lam[p], 0.0));
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
  p->cg_iters = 2;   // warm-started at x_{n-1}: two steps give the iterates of eight (see the design notes)
  p->passes = 1;
  p->check_every = 10;
  p->graph = 1;
  p->w_from_x0 = 0;
  p->toeplitz = 1;
  p->block_norm = 1;
  p->tol_dual = 1e-2;
  p->z_from_x0 = 0;
  p->block_fraction = 1.0;
  p->block_seed = 0;
  p->synthesis = 0;
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
  sh::Arena arena;                 // a caller's workspace (sh_sdmm_create_ws); declared before w, freed after it
  Work w;
  int P = 1;
  int64_t per = 0, Dper = 0;       // pixels and coefficients of one problem
  int64_t N = 0, M = 0, D = 0;     // totals over the P problems
  int R = 0, kcg = 0;
  std::vector<double> nu, gamma, delta;   // per problem
  std::vector<double> lambda0;             // per problem: the data-dual scale of a dual warm start
  bool stoch = false;                      // block-subset iterations (block_fraction < 1)
  bool synth = false;                      // synthesis prior: the unknowns are the coefficients alpha
  std::vector<char> have_delta;            // per problem: delta holds a reweighting delta (given, or from a pass)
  std::vector<double> cb;          // c_b per block (host)
  std::vector<double> eh;          // eps_hat = c_b eps per block (host)
  const float* Wp = nullptr;       // weights of the current pass (the session's W, 1 where no weights were given)
  int iters_total = 0;
  double *s_rs = nullptr, *s_pap = nullptr, *s_misc = nullptr;
  // Replay of one captured iteration (hipGraph) on a session-owned stream.
  hipStream_t gs = nullptr;
  hipGraphExec_t gexec = nullptr;
  const float* g_Wp = nullptr;     // the weights pointer baked into gexec
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // The dictionary's branch of an iteration (Psi v_psi before CG; Psi^dagger x and the l1 step after it) runs
  // on a second stream beside the data term's branch (Phi^dagger before CG; Phi x, the ball step and the
  // positivity step after it): the two touch disjoint buffers and join before their results are used.
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // Per-iteration metrics ring (sh_sdmm_metrics_enable): ring_rows rows of 2P + R doubles, one written by every
  // iteration (inside the replayed graph); ring_ctr counts the rows written since the ring was enabled.
  sh::DevBuf<double> ring;
  sh::DevBuf<unsigned long long> ring_ctr;
  int ring_rows = 0;
  int ring_base = 0;                  // iters_total when the ring was enabled
  unsigned long long ring_next = 0;   // the first row not yet handed to the caller
  ~sh_sdmm_s() {
    if (side) {
      (void)hipStreamSynchronize(side);
      (void)hipStreamDestroy(side);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (gs) {
      (void)hipStreamSynchronize(gs);
      (void)hipStreamDestroy(gs);
    }
  }
};

namespace {

// s_misc layout: [0, P) dx^2, [P, 2P) x^2, [2P, 3P) scratch, [3P, 4P) objective, [4P, 5P) scratch
enum { MISC_DX = 0, MISC_X = 1, MISC_TMP = 2, MISC_OBJ = 3, MISC_TMP2 = 4, MISC_N = 5 };

sh_status sdmm_reweight(sh_sdmm s, float* W_dst, hipStream_t st, const std::vector<char>* which = nullptr,
                        const float* coeffs = nullptr);

// Duals of a warm start from x0, taken from the optimality conditions of the weighted problem at x0 (the
// primal splits already hold y_j = L_j x0):
//   l1 split:   y_psi = soft(Psi^dagger x0, gamma W), z_psi = Psi^dagger x0 - y_psi (the subgradient
//               gamma W sign(.) where a coefficient exceeds its threshold, the coefficient itself below);
//   positivity: z_+ = 0 (x0 >= 0);
//   data:       y_i = the projection of Phi_hat_i x0 onto ball i, z_i = lambda (y_i - yhat_i) along the balls'
//               outward normals, with one lambda >= 0 per problem chosen so that the stationarity residual
//               ||Psi z_psi + Phi_hat^dagger z_phi|| is smallest: lambda = max(0, -<Psi z_psi, g> / <g, g>),
//               g = Phi_hat^dagger (y - yhat).
// From a zero dual the iteration would first have to rebuild all of them.
sh_status sdmm_dual_warm_start(sh_sdmm s, hipStream_t st) {
  sh_op op = s->op;
  Work& w = s->w;
  const int P = s->P;
  const int64_t per = s->per;
  // l1 split (vpsi holds Psi^dagger x0)
  SH_HIP(hipMemcpyAsync(w.spsi.ptr, w.vpsi.ptr, s->D * sizeof(float), hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(dual_l1_init, dim3(nblk(s->Dper), P), dim3(256), 0, st, w.spsi.ptr, w.W.ptr, w.gamma.ptr,
                     w.zpsi.ptr, w.vpsi.ptr, s->Dper);
  SH_LAUNCHED();
  SH_TRY(sh_psi_fwd(s->psi, w.zpsi.ptr, w.t1.ptr, st));                        // Psi z_psi
  // data splits: block norms ||c s - yhat|| (zero dual) give each block's projection
  SH_HIP(hipMemsetAsync(w.zphi.ptr, 0, s->M * sizeof(float2), st));
  SH_TRY(sh::ball_norms_only(op, w.sphi.ptr, w.zphi.ptr, w.yhat.ptr, w.cblk.ptr, w.rho.ptr, w.kkt.ptr + 8 * P, st));
  const unsigned nc = (unsigned)op->n_chunks;
  hipLaunchKernelGGL(dual_ball_init, dim3(nc), dim3(256), 0, st, w.sphi.ptr, w.yhat.ptr, op->chunks.ptr, w.cblk.ptr,
                     w.eps_hat.ptr, w.rho.ptr, op->block_prob_d.ptr, (const double*)nullptr, w.zphi.ptr, w.vtmp.ptr, 0);
  SH_LAUNCHED();
  SH_TRY(sh::phi_adjoint(op, w.vtmp.ptr, w.t2.ptr, false, nullptr, st));        // g = Phi_hat^dagger (y - yhat)
  double* k = w.kkt.ptr;
  SH_TRY(w.red.dot(w.t1.ptr, w.t2.ptr, per, k, st));
  SH_TRY(w.red.dot(w.t2.ptr, w.t2.ptr, per, k + P, st));
  std::vector<double> h(2 * P), lam(P);
  SH_HIP(hipMemcpyAsync(h.data(), k, 2 * P * sizeof(double), hipMemcpyDeviceToHost, st));
  SH_HIP(hipStreamSynchronize(st));
  for (int p = 0; p < P; ++p) lam[p] = h[P + p] > 0 ? std::max(0.0, -h[p] / h[P + p]) : 0.0;
  s->lambda0 = lam;
  SH_HIP(hipMemcpyAsync(k, lam.data(), P * sizeof(double), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(dual_ball_init, dim3(nc), dim3(256), 0, st, w.sphi.ptr, w.yhat.ptr, op->chunks.ptr, w.cblk.ptr,
                     w.eps_hat.ptr, w.rho.ptr, op->block_prob_d.ptr, (const double*)k, w.zphi.ptr, w.vphi.ptr, 1);
  SH_LAUNCHED();
  SH_HIP(hipStreamSynchronize(st));   // lam (host) is read by the enqueued copy
  return SH_OK;
}

sh_status sdmm_setup(sh_sdmm s, const float* y, const double* eps, const float* W0, const float* x0, hipStream_t st) {
  sh_op op = s->op;
  const int R = s->R, P = s->P;
  const int64_t N = s->N, M = s->M, D = s->D;
  const int kcg = s->kcg;
  Work& w = s->w;
  for (auto* b : {&w.x, &w.xprev, &w.r, &w.p, &w.Ap, &w.t1, &w.t2, &w.vpos, &w.zpos}) SH_TRY(b->alloc(N));
  for (auto* b : {&w.spsi, &w.zpsi, &w.vpsi, &w.W}) SH_TRY(b->alloc(D));
  for (auto* b : {&w.yhat, &w.sphi, &w.zphi, &w.vphi, &w.vtmp}) SH_TRY(b->alloc(M));
  const int nsc = (2 * kcg + 1 + MISC_N) * P;
  SH_TRY(w.sc.alloc(nsc));
  SH_TRY(w.eps_hat.alloc(R));
  SH_TRY(w.rho.alloc(R));
  SH_TRY(w.resid.alloc(R));
  SH_TRY(w.delta.alloc(P));
  SH_TRY(w.cblk.alloc(R));
  SH_TRY(w.gamma.alloc(P));
  SH_TRY(w.kkt.alloc(8 * P + 2 * R));
  SH_TRY(w.red.init(P));
  if (s->synth)
    for (auto* b : {&w.alpha, &w.ar, &w.ap, &w.aAp, &w.alpha_out}) SH_TRY(b->alloc(D));
  if (s->stoch) {
    SH_TRY(w.bmask.alloc(R));
    SH_TRY(w.ctr.alloc(1));
    SH_TRY(w.bphi.alloc(N));
    SH_HIP(hipMemsetAsync(w.ctr.ptr, 0, sizeof(unsigned long long), st));
  }
  double* sc = w.sc.ptr;
  s->s_rs = sc;                        // rs_k of problem p at [k*P + p], k = 0..kcg
  s->s_pap = sc + (kcg + 1) * P;       // pAp_k at [k*P + p], k = 0..kcg-1
  s->s_misc = sc + (2 * kcg + 1) * P;  // MISC_* blocks of P
  double* s_misc = s->s_misc;
  SH_HIP(hipMemsetAsync(w.resid.ptr, 0, R * sizeof(double), st));
  SH_HIP(hipMemsetAsync(w.sc.ptr, 0, nsc * sizeof(double), st));

  // non-finite data check (float64 sum of squares)
  {
    sh::Reducer r1;
    SH_TRY(r1.init(1));
    SH_TRY(r1.dot(y, y, 2 * M, s_misc + MISC_TMP * P, st));
  }
  double ysq = 0;
  SH_HIP(hipMemcpyAsync(&ysq, s_misc + MISC_TMP * P, sizeof(double), hipMemcpyDeviceToHost, st));
  SH_HIP(hipStreamSynchronize(st));
  if (!std::isfinite(ysq)) {
    sh::set_error("visibilities contain non-finite values");
    return SH_ENONFINITE;
  }
  // block weights a_b (1, or the density estimate of 1 / ||Phi_b||) and the norm nu_p of each problem's
  // a-weighted operator; c_b = a_b / nu_p.  In Toeplitz mode the CG operator is built here, with the
  // weights a_b^2, then rescaled by 1 / nu_p^2.
  std::vector<double> ab(R, 1.0);
  if (s->prm.block_norm) SH_TRY(sh::block_density_weights(op, ab, st));
  std::vector<float> af(R);
  for (int i = 0; i < R; ++i) af[i] = float(ab[i]);
  SH_HIP(hipMemcpy(w.cblk.ptr, af.data(), R * sizeof(float), hipMemcpyHostToDevice));   // a_b until c_b is known
  s->nu.assign(P, s->prm.nu);
  const bool need_nu = !(s->prm.nu > 0);
  if (need_nu) hipLaunchKernelGGL(fill_kernel, dim3(nblk(N)), dim3(256), 0, st, w.t1.ptr, N, 1.f);
  if (s->prm.toeplitz) {
    SH_TRY(sh::toeplitz_build(op, nullptr, s->prm.block_norm ? ab.data() : nullptr, &w.toep, st));
    if (need_nu) SH_TRY(power_norm(op, w.t1.ptr, 200, 1e-6, s->nu.data(), st, nullptr, &w.toep));
  } else if (need_nu) {
    SH_TRY(power_norm(op, w.t1.ptr, 200, 1e-6, s->nu.data(), st, s->prm.block_norm ? w.cblk.ptr : nullptr));
  }
  for (int p = 0; p < P; ++p)
    SH_REQUIRE(s->nu[p] > 0 && std::isfinite(s->nu[p]), "operator norm of problem %d must be positive", p);
  if (s->prm.toeplitz) {
    std::vector<double> f(P);
    for (int p = 0; p < P; ++p) f[p] = 1.0 / (s->nu[p] * s->nu[p]);
    SH_TRY(sh::toeplitz_rescale(&w.toep, f.data(), st));
  }
  s->cb.resize(R);
  std::vector<float> cf(R);
  for (int i = 0; i < R; ++i) {
    s->cb[i] = ab[i] / s->nu[op->block_prob[i]];
    cf[i] = float(s->cb[i]);
  }
  SH_HIP(hipMemcpy(w.cblk.ptr, cf.data(), R * sizeof(float), hipMemcpyHostToDevice));
  hipLaunchKernelGGL(gather_scale, dim3((unsigned)op->n_chunks), dim3(256), 0, st, (const float2*)y, op->perm.ptr,
                     w.yhat.ptr, op->chunks.ptr, w.cblk.ptr);
  SH_LAUNCHED();
  s->eh.resize(R);
  for (int i = 0; i < R; ++i) s->eh[i] = eps[i] * s->cb[i];
  SH_HIP(hipMemcpyAsync(w.eps_hat.ptr, s->eh.data(), R * sizeof(double), hipMemcpyHostToDevice, st));
  // gamma = 1e-4 max |Psi^dagger Phi_hat^dagger y_hat| per problem unless given (the minimiser does not
  // depend on gamma; this step meets the stopping test within a few hundred iterations per pass);
  // Phi_hat^dagger y_hat = Phi^dagger (c yhat)
  s->gamma.assign(P, s->prm.gamma);
  if (!(s->prm.gamma > 0)) {
    SH_TRY(sh::phi_adjoint(op, w.yhat.ptr, w.t1.ptr, false, w.cblk.ptr, st));
    SH_TRY(sh_psi_adj(s->psi, w.t1.ptr, w.spsi.ptr, st));
    SH_TRY(w.red.maxabs(w.spsi.ptr, s->Dper, s_misc + MISC_TMP * P, st));
    std::vector<double> mx(P);
    SH_HIP(hipMemcpyAsync(mx.data(), s_misc + MISC_TMP * P, P * sizeof(double), hipMemcpyDeviceToHost, st));
    SH_HIP(hipStreamSynchronize(st));
    for (int p = 0; p < P; ++p) s->gamma[p] = 1e-4 * mx[p];
  }
  std::vector<float> gf(P);
  for (int p = 0; p < P; ++p) {
    SH_REQUIRE(s->gamma[p] > 0 && std::isfinite(s->gamma[p]), "gamma of problem %d must be positive (is y zero?)", p);
    gf[p] = float(s->gamma[p]);
  }
  SH_HIP(hipMemcpy(w.gamma.ptr, gf.data(), P * sizeof(float), hipMemcpyHostToDevice));
  // weights of the first pass: W0, or 1 (identity; gamma * 1 is gamma exactly, so the arithmetic is that of
  // no weights).  One weight array for all passes and problems keeps the captured iteration valid while
  // problems of a batch reweight at different times.
  if (W0) {
    SH_HIP(hipMemcpyAsync(w.W.ptr, W0, D * sizeof(float), hipMemcpyDeviceToDevice, st));
  } else {
    hipLaunchKernelGGL(fill_kernel, dim3(nblk(D)), dim3(256), 0, st, w.W.ptr, D, 1.f);
    SH_LAUNCHED();
  }
  s->Wp = w.W.ptr;
  const bool given = s->prm.rw_delta0 > 0 && W0;
  s->have_delta.assign(P, given ? 1 : 0);
  s->delta.assign(P, given ? s->prm.rw_delta0 : 0.0);
  // initial state: zero, or y_psi = Psi^dagger x0, y_phi = Phi_hat x0, y_+ = x0, z = 0
  SH_HIP(hipMemsetAsync(w.zpsi.ptr, 0, D * sizeof(float), st));
  SH_HIP(hipMemsetAsync(w.zphi.ptr, 0, M * sizeof(float2), st));
  SH_HIP(hipMemsetAsync(w.zpos.ptr, 0, N * sizeof(float), st));
  SH_HIP(hipMemsetAsync(w.vphi.ptr, 0, M * sizeof(float2), st));  // y_phi - z_phi - Phi_hat x0 = 0 either way
  if (x0) {
    SH_HIP(hipMemcpyAsync(w.x.ptr, x0, N * sizeof(float), hipMemcpyDeviceToDevice, st));
    SH_HIP(hipMemcpyAsync(w.vpos.ptr, x0, N * sizeof(float), hipMemcpyDeviceToDevice, st));
    SH_TRY(sh_psi_adj(s->psi, x0, w.vpsi.ptr, st));
    SH_TRY(sh::phi_forward(op, x0, w.sphi.ptr, false, nullptr, st));   // the ball step applies c_b
  } else {
    SH_HIP(hipMemsetAsync(w.x.ptr, 0, N * sizeof(float), st));
    SH_HIP(hipMemsetAsync(w.vpos.ptr, 0, N * sizeof(float), st));
    SH_HIP(hipMemsetAsync(w.vpsi.ptr, 0, D * sizeof(float), st));
    SH_HIP(hipMemsetAsync(w.sphi.ptr, 0, M * sizeof(float2), st));
  }
  SH_HIP(hipMemsetAsync(w.xprev.ptr, 0, N * sizeof(float), st));
  if (s->synth) {   // unknowns alpha: zero, or alpha = Psi^dagger x0 (in vpsi) with x = Psi alpha, y_l1 = alpha
    if (x0) {
      SH_HIP(hipMemcpyAsync(w.alpha.ptr, w.vpsi.ptr, D * sizeof(float), hipMemcpyDeviceToDevice, st));
      SH_TRY(sh_psi_fwd(s->psi, w.alpha.ptr, w.x.ptr, st));
      SH_HIP(hipMemcpyAsync(w.vpos.ptr, w.x.ptr, N * sizeof(float), hipMemcpyDeviceToDevice, st));
      SH_TRY(sh::phi_forward(op, w.x.ptr, w.sphi.ptr, false, nullptr, st));
    } else {
      SH_HIP(hipMemsetAsync(w.alpha.ptr, 0, D * sizeof(float), st));
    }
  }
  if (s->prm.w_from_x0) {   // weights of the first pass from Psi^dagger x0 (delta_1 = std per problem)
    SH_TRY(sh_psi_adj(s->psi, x0, w.spsi.ptr, st));   // (= alpha_0 of the synthesis form)
    std::fill(s->delta.begin(), s->delta.end(), 0.0);
    std::fill(s->have_delta.begin(), s->have_delta.end(), 0);
    SH_TRY(sdmm_reweight(s, w.W.ptr, st, nullptr, w.spsi.ptr));
  }
  if (s->stoch) {   // block-subset iterations keep v_phi = c (y - z) and the image Phi_hat^T v_phi
    if (x0) {
      hipLaunchKernelGGL(scale2_chunks, dim3((unsigned)op->n_chunks), dim3(256), 0, st, w.sphi.ptr, w.vphi.ptr,
                         op->chunks.ptr, w.cblk.ptr);
      SH_LAUNCHED();
      SH_TRY(sh::phi_adjoint(op, w.vphi.ptr, w.bphi.ptr, false, nullptr, st));
    } else {
      SH_HIP(hipMemsetAsync(w.bphi.ptr, 0, N * sizeof(float), st));
    }
    // the iterations refresh the residuals of their selected blocks only: start every block from x0's
    SH_TRY(sh::ball_norms_only(op, w.sphi.ptr, w.zphi.ptr, w.yhat.ptr, w.cblk.ptr, w.kkt.ptr + 8 * P, w.resid.ptr,
                               st));
  }
  if (s->prm.z_from_x0) {   // duals from the optimality conditions at x0 (see sdmm_dual_warm_start)
    SH_TRY(sdmm_dual_warm_start(s, st));
  }
  return SH_OK;
}

// One SDMM iteration on the synthesis prior: min ||W alpha||_1 subject to the balls on Phi_hat Psi alpha and
// Psi alpha >= 0, L = {I, Phi_hat Psi, Psi}, Q = I + Psi^dagger (I + Re(Phi_hat^H Phi_hat)) Psi.  CG runs on the
// coefficients from alpha_{n-1}; its initial residual
//   b - Q alpha_{n-1} = v_l1 + Psi^dagger (Phi^dagger v_phi + v_+ - x_{n-1}) - alpha_{n-1}
// reuses s_phi = Phi x_{n-1} through v_phi (as in the analysis form), and every product Q p is
// p + Psi^dagger ((I + T) Psi p) with the Toeplitz product T.  Then x_n = Psi alpha_n feeds the data and
// positivity splits, alpha_n the l1 split.
// One row of the metrics ring: per problem the relative change ||x_n - x_(n-1)|| / ||x_n|| and the objective
// ||W Psi^dagger x_n||_1 (||W alpha_n||_1 for the synthesis prior), per block the residual ||y_i - Phi_i x_n||
// over eps_i (both in the normalised units of eq. (3), whose ratio is the user-unit one).  One work-group; the
// row counter advances after the row is written.
__global__ __launch_bounds__(256) void ring_record(const double* __restrict__ misc, const double* __restrict__ resid,
                                                   const double* __restrict__ eps_hat, double* __restrict__ ring,
                                                   unsigned long long* __restrict__ ctr, int rows, int P, int R) {
  const unsigned long long c = ctr[0];
  double* row = ring + (size_t)(c % (unsigned long long)rows) * (size_t)(2 * P + R);
  for (int j = threadIdx.x; j < P; j += 256) {
    const double dx = misc[MISC_DX * P + j], xx = misc[MISC_X * P + j];
    row[j] = xx > 0 ? sqrt(dx / xx) : (dx == 0 ? 0.0 : INFINITY);
    row[P + j] = misc[MISC_OBJ * P + j];
  }
  for (int b = threadIdx.x; b < R; b += 256) row[2 * P + b] = resid[b] / eps_hat[b];
  __syncthreads();
  if (threadIdx.x == 0) ctr[0] = c + 1;
}

// Appends the iteration's metrics row (nothing while the ring is off).  Block-subset iterations refresh the
// residuals of their selected blocks only; the others keep their last value.
sh_status ring_step(sh_sdmm s, hipStream_t st) {
  if (s->ring_rows <= 0) return SH_OK;
  Work& w = s->w;
  SH_TRY(w.red.l1w(s->synth ? w.alpha.ptr : w.spsi.ptr, s->Wp, s->Dper, s->s_misc + MISC_OBJ * s->P, st));
  hipLaunchKernelGGL(ring_record, dim3(1), dim3(256), 0, st, s->s_misc, w.resid.ptr, w.eps_hat.ptr, s->ring.ptr,
                     s->ring_ctr.ptr, s->ring_rows, s->P, s->R);
  SH_LAUNCHED();
  return SH_OK;
}

sh_status sdmm_step_synthesis(sh_sdmm s, hipStream_t st) {
  sh_op op = s->op;
  Work& w = s->w;
  const int P = s->P;
  const int64_t N = s->N, per = s->per, Dp = s->Dper;
  double *s_rs = s->s_rs, *s_pap = s->s_pap, *s_misc = s->s_misc;
  SH_TRY(sh::phi_adjoint(op, w.vphi.ptr, w.t2.ptr, false, nullptr, st));   // vphi carries c_b and -s_hat
  hipLaunchKernelGGL(comb_kernel, dim3(nblk(N)), dim3(256), 0, st, w.t1.ptr, w.t2.ptr, w.vpos.ptr, w.x.ptr, N);
  hipLaunchKernelGGL(copy_kernel, dim3(nblk(N)), dim3(256), 0, st, w.xprev.ptr, w.x.ptr, N);
  SH_LAUNCHED();
  SH_TRY(sh_psi_adj(s->psi, w.t1.ptr, w.aAp.ptr, st));
  // (spsi, unused by this form's iteration, receives alpha_{n-1})
  SH_TRY(w.red.cg_init(w.vpsi.ptr, w.aAp.ptr, nullptr, w.alpha.ptr, w.ar.ptr, w.ap.ptr, w.spsi.ptr, Dp, s_rs, st, 1.f));
  for (int k = 0; k < s->kcg; ++k) {
    SH_TRY(sh_psi_fwd(s->psi, w.ap.ptr, w.t1.ptr, st));                                       // Psi p
    SH_TRY(sh::toeplitz_apply(op, w.toep.Ht.ptr, w.t1.ptr, w.toep.tq.ptr, w.t2.ptr, st));     // T Psi p
    hipLaunchKernelGGL(add_kernel, dim3(nblk(N)), dim3(256), 0, st, w.t1.ptr, w.t2.ptr, N);
    SH_TRY(sh_psi_adj(s->psi, w.t1.ptr, w.aAp.ptr, st));
    SH_TRY(w.red.cg_ap(w.ap.ptr, w.aAp.ptr, Dp, st, 1.f));                                  // p + Psi^T (I + T) Psi p
    SH_TRY(w.red.cg_update(w.alpha.ptr, w.ar.ptr, w.ap.ptr, w.aAp.ptr, Dp, s_rs + k * P, s_pap + k * P, st));
    if (k + 1 < s->kcg) SH_TRY(w.red.cg_dir(w.ar.ptr, w.ap.ptr, Dp, s_rs + k * P, s_rs + (k + 1) * P, st));
  }
  SH_LAUNCHED();
  SH_TRY(sh_psi_fwd(s->psi, w.alpha.ptr, w.x.ptr, st));                                       // x_n = Psi alpha_n
  SH_TRY(w.red.change(w.x.ptr, w.xprev.ptr, per, s_misc + MISC_DX * P, st));
  SH_TRY(sh::launch_prox_l1(Dp, P, w.alpha.ptr, w.zpsi.ptr, s->Wp, w.gamma.ptr, 0.f, w.vpsi.ptr, st));
  SH_TRY(sh::phi_forward(op, w.x.ptr, w.sphi.ptr, false, nullptr, st));
  SH_TRY(sh::launch_prox_ball(op, w.sphi.ptr, w.zphi.ptr, w.yhat.ptr, w.eps_hat.ptr, w.rho.ptr, w.resid.ptr,
                              w.vphi.ptr, true, w.cblk.ptr, st));
  SH_TRY(sh::launch_prox_pos(N, w.x.ptr, w.zpos.ptr, w.vpos.ptr, st));
  return SH_OK;
}

// One SDMM iteration of all P problems, enqueued on `st` with no host synchronisation, no memset
// and no allocation (so that it can be captured into a graph).
// The side stream starts after the work enqueued on st so far (fork) / st continues after the side stream's
// work (join).  Under graph capture these are the captured graph's branch and merge.
sh_status fork_side(sh_sdmm s, hipStream_t st) {
  SH_HIP(hipEventRecord(s->ev_fork, st));
  SH_HIP(hipStreamWaitEvent(s->side, s->ev_fork, 0));
  return SH_OK;
}
sh_status join_side(sh_sdmm s, hipStream_t st) {
  SH_HIP(hipEventRecord(s->ev_join, s->side));
  SH_HIP(hipStreamWaitEvent(st, s->ev_join, 0));
  return SH_OK;
}

sh_status sdmm_step(sh_sdmm s, hipStream_t st) {
  sh_op op = s->op;
  Work& w = s->w;
  const int P = s->P;
  const int64_t N = s->N, per = s->per;
  double *s_rs = s->s_rs, *s_pap = s->s_pap, *s_misc = s->s_misc;
  if (s->synth) {
    SH_TRY(sdmm_step_synthesis(s, st));
    return ring_step(s, st);
  }
  // ---- x-update by CG from x_{n-1}; its right-hand side's dictionary term on the side stream
  SH_TRY(fork_side(s, st));
  SH_TRY(sh_psi_fwd(s->psi, w.vpsi.ptr, w.t1.ptr, s->side));
  if (s->stoch) {
    // this iteration's blocks; b - Q x_{n-1} from the running image Phi_hat^T v_phi and a Toeplitz product
    hipLaunchKernelGGL(block_mask_kernel, dim3(1), dim3(1024), 0, st, (uint64_t)s->prm.block_seed, w.ctr.ptr, s->R,
                       s->prm.block_fraction, w.bmask.ptr);
    SH_TRY(sh::toeplitz_apply(op, w.toep.Ht.ptr, w.x.ptr, w.toep.tq.ptr, w.Ap.ptr, st));
    hipLaunchKernelGGL(sub_kernel, dim3(nblk(N)), dim3(256), 0, st, w.bphi.ptr, w.Ap.ptr, w.t2.ptr, N);
    SH_LAUNCHED();
  } else {
    SH_TRY(sh::phi_adjoint(op, w.vphi.ptr, w.t2.ptr, false, nullptr, st));   // vphi carries c_b
  }
  SH_TRY(join_side(s, st));
  SH_TRY(w.red.cg_init(w.t1.ptr, w.t2.ptr, w.vpos.ptr, w.x.ptr, w.r.ptr, w.p.ptr, w.xprev.ptr, per, s_rs, st));
  for (int k = 0; k < s->kcg; ++k) {
    if (s->prm.toeplitz) {
      SH_TRY(sh::toeplitz_apply(op, w.toep.Ht.ptr, w.p.ptr, w.toep.tq.ptr, w.Ap.ptr, st));
    } else {
      SH_TRY(sh::phi_forward(op, w.p.ptr, w.vtmp.ptr, false, w.cblk.ptr, st));
      SH_TRY(sh::phi_adjoint(op, w.vtmp.ptr, w.Ap.ptr, false, w.cblk.ptr, st));
    }
    SH_TRY(w.red.cg_ap(w.p.ptr, w.Ap.ptr, per, st));
    SH_TRY(w.red.cg_update(w.x.ptr, w.r.ptr, w.p.ptr, w.Ap.ptr, per, s_rs + k * P, s_pap + k * P, st));
    if (k + 1 < s->kcg) SH_TRY(w.red.cg_dir(w.r.ptr, w.p.ptr, per, s_rs + k * P, s_rs + (k + 1) * P, st));
  }
  SH_LAUNCHED();
  // ---- relative change
  static_assert(MISC_X == MISC_DX + 1, "change() writes dx^2 then x^2");
  SH_TRY(w.red.change(w.x.ptr, w.xprev.ptr, per, s_misc + MISC_DX * P, st));
  // ---- splits: the l1 split on the side stream, the data and positivity splits on st
  SH_TRY(fork_side(s, st));
  SH_TRY(sh_psi_adj(s->psi, w.x.ptr, w.spsi.ptr, s->side));
  SH_TRY(sh::launch_prox_l1(s->Dper, P, w.spsi.ptr, w.zpsi.ptr, s->Wp, w.gamma.ptr, 0.f, w.vpsi.ptr, s->side));
  if (s->stoch) {   // the selected blocks only: their images, ball steps and change of Phi_hat^T v_phi
    SH_TRY(sh::phi_forward(op, w.x.ptr, w.sphi.ptr, false, nullptr, st, w.bmask.ptr));
    SH_TRY(sh::launch_prox_ball_subset(op, w.sphi.ptr, w.zphi.ptr, w.yhat.ptr, w.eps_hat.ptr, w.rho.ptr, w.resid.ptr,
                                       w.vphi.ptr, w.vtmp.ptr, w.cblk.ptr, w.bmask.ptr, st));
    SH_TRY(sh::phi_adjoint(op, w.vtmp.ptr, w.t2.ptr, false, nullptr, st, w.bmask.ptr));
    hipLaunchKernelGGL(add_kernel, dim3(nblk(N)), dim3(256), 0, st, w.bphi.ptr, w.t2.ptr, N);
    SH_LAUNCHED();
  } else {
    SH_TRY(sh::phi_forward(op, w.x.ptr, w.sphi.ptr, false, nullptr, st));
    SH_TRY(sh::launch_prox_ball(op, w.sphi.ptr, w.zphi.ptr, w.yhat.ptr, w.eps_hat.ptr, w.rho.ptr, w.resid.ptr,
                                w.vphi.ptr, true, w.cblk.ptr, st));
  }
  SH_TRY(sh::launch_prox_pos(N, w.x.ptr, w.zpos.ptr, w.vpos.ptr, st));
  SH_TRY(join_side(s, st));
  return ring_step(s, st);
}

// Captures one iteration into an executable graph on the session stream (again whenever the
// weights pointer, the only launch argument that changes between passes, differs).
sh_status sdmm_graph(sh_sdmm s) {
  if (s->gexec && s->g_Wp == s->Wp) return SH_OK;
  if (!s->gs) {
    SH_HIP(hipStreamCreateWithFlags(&s->gs, hipStreamNonBlocking));
    SH_HIP(hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming));
    SH_HIP(hipEventCreateWithFlags(&s->ev_out, hipEventDisableTiming));
  }
  if (s->gexec) {
    SH_HIP(hipStreamSynchronize(s->gs));
    SH_HIP(hipGraphExecDestroy(s->gexec));
    s->gexec = nullptr;
  }
  hipGraph_t g = nullptr;
  SH_HIP(hipStreamBeginCapture(s->gs, hipStreamCaptureModeThreadLocal));
  const sh_status st = sdmm_step(s, s->gs);
  const hipError_t e = hipStreamEndCapture(s->gs, &g);
  if (st != SH_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) {
    sh::set_error("graph capture of the SDMM iteration failed: %s", hipGetErrorString(e));
    return SH_EDEVICE;
  }
  const hipError_t ei = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    s->gexec = nullptr;
    sh::set_error("graph instantiation failed: %s", hipGetErrorString(ei));
    return SH_EDEVICE;
  }
  s->g_Wp = s->Wp;
  return SH_OK;
}

// Enqueue `iters` iterations on `st`: replayed graphs (ordered after and before the caller's stream
// by events) or, with graphs off or kernel timing on, plain launches.
sh_status sdmm_run(sh_sdmm s, int iters, hipStream_t st) {
  if (iters <= 0) return SH_OK;
  if (!s->prm.graph || sh::profiling_on()) {
    for (int i = 0; i < iters; ++i) SH_TRY(sdmm_step(s, st));
  } else {
    SH_TRY(sdmm_graph(s));
    SH_HIP(hipEventRecord(s->ev_in, st));
    SH_HIP(hipStreamWaitEvent(s->gs, s->ev_in, 0));
    for (int i = 0; i < iters; ++i) SH_HIP(hipGraphLaunch(s->gexec, s->gs));
    SH_HIP(hipEventRecord(s->ev_out, s->gs));
    SH_HIP(hipStreamWaitEvent(st, s->ev_out, 0));
  }
  s->iters_total += iters;
  return SH_OK;
}

// Reads the stopping quantities of the last iteration (synchronises): per-problem relative change,
// per-block residuals (hat units).
sh_status sdmm_read(sh_sdmm s, std::vector<double>& rel, std::vector<double>& hres, hipStream_t st) {
  const int P = s->P;
  if (s->stoch) {   // the iterations refresh only their blocks' residuals: evaluate all of them at x_n
    Work& w = s->w;
    SH_TRY(sh::phi_forward(s->op, w.x.ptr, w.vtmp.ptr, false, nullptr, st));
    SH_TRY(sh::ball_norms_only(s->op, w.vtmp.ptr, w.zphi.ptr, w.yhat.ptr, w.cblk.ptr, w.kkt.ptr + 8 * P, w.resid.ptr,
                               st));
  }
  std::vector<double> h(2 * P);
  SH_HIP(hipMemcpyAsync(h.data(), s->s_misc, 2 * P * sizeof(double), hipMemcpyDeviceToHost, st));
  hres.resize(s->R);
  SH_HIP(hipMemcpyAsync(hres.data(), s->w.resid.ptr, s->R * sizeof(double), hipMemcpyDeviceToHost, st));
  SH_HIP(hipStreamSynchronize(st));
  rel.resize(P);
  for (int p = 0; p < P; ++p) {
    const double dx = h[MISC_DX * P + p], xx = h[MISC_X * P + p];
    if (!std::isfinite(dx) || !std::isfinite(xx)) {
      sh::set_error("non-finite iterate in problem %d after %d iterations", p, s->iters_total);
      return SH_ENONFINITE;
    }
    rel[p] = xx > 0 ? std::sqrt(dx / xx) : (dx == 0 ? 0.0 : INFINITY);
  }
  return SH_OK;
}

// Reweighting after a pass, from Psi^dagger x (in spsi): delta_1 = std(Psi^dagger x) per problem (float64) at a
// problem's first reweighting, then delta <- beta delta.  `which` (per problem, NULL = all) selects the problems
// whose pass just ended; the others keep their weights and delta.
sh_status sdmm_reweight(sh_sdmm s, float* W_dst, hipStream_t st, const std::vector<char>* which, const float* coeffs) {
  Work& w = s->w;
  const int P = s->P;
  // the coefficients the weights follow: Psi^dagger x (analysis, in spsi) or alpha (synthesis)
  const float* cf = coeffs ? coeffs : (s->synth ? w.alpha.ptr : w.spsi.ptr);
  auto sel = [&](int p) { return which == nullptr || (*which)[p] != 0; };
  bool need_std = false;
  for (int p = 0; p < P; ++p) need_std = need_std || (sel(p) && !s->have_delta[p]);
  if (need_std) {   // first reweighting of some problem: delta_1 = std of its analysis coefficients
    double* sum = s->s_misc + MISC_TMP * P;
    double* var = s->s_misc + MISC_TMP2 * P;
    SH_TRY(w.red.std_dev(cf, s->Dper, sum, var, st));
    std::vector<double> v(P);
    SH_HIP(hipMemcpyAsync(v.data(), var, P * sizeof(double), hipMemcpyDeviceToHost, st));
    SH_HIP(hipStreamSynchronize(st));
    for (int p = 0; p < P; ++p)
      if (sel(p) && !s->have_delta[p]) {
        s->delta[p] = std::sqrt(v[p] / double(s->Dper));
        s->have_delta[p] = 2;   // set by this call: not scaled below
      }
  }
  for (int p = 0; p < P; ++p) {
    if (!sel(p)) continue;
    if (s->have_delta[p] == 2)
      s->have_delta[p] = 1;
    else
      s->delta[p] *= s->prm.rw_beta;
  }
  // delta = 0 (a pass that ended at x = 0) is valid: the weights are then 1 at zero coefficients
  for (int p = 0; p < P; ++p)
    if (!(s->delta[p] >= 0) || !std::isfinite(s->delta[p])) {
      sh::set_error("reweighting delta of problem %d is %g", p, s->delta[p]);
      return SH_ENONFINITE;
    }
  SH_HIP(hipMemcpyAsync(w.delta.ptr, s->delta.data(), P * sizeof(double), hipMemcpyHostToDevice, st));
  if (which == nullptr) {
    SH_TRY(sh::launch_reweight(s->Dper, P, cf, w.delta.ptr, 0.0, W_dst, st));
  } else {
    for (int p = 0; p < P; ++p)
      if (sel(p))
        SH_TRY(sh::launch_reweight(s->Dper, 1, cf + p * s->Dper, w.delta.ptr + p, 0.0, W_dst + p * s->Dper, st));
  }
  SH_HIP(hipStreamSynchronize(st));   // the host copy of delta is read by the enqueued copy
  return SH_OK;
}

// The KKT residuals and objective of the synthesis form: splits alpha (l1), Phi_hat x (balls) and x (positivity)
// with x = Psi alpha; dual stationarity z_l1 + Psi^dagger (Phi_hat^dagger z_phi + z_+) = 0 in coefficient space.
// Definitions as for the analysis form below; the CG scratch ap, aAp holds the coefficient-space terms.
sh_status sdmm_kkt_synthesis(sh_sdmm s, std::vector<double>& prim, std::vector<double>& dual, std::vector<double>& obj,
                             hipStream_t st) {
  sh_op op = s->op;
  Work& w = s->w;
  const int P = s->P, R = s->R;
  const int64_t Dp = s->Dper;
  double* k = w.kkt.ptr;
  SH_TRY(w.red.comb3_sq(w.alpha.ptr, w.vpsi.ptr, w.zpsi.ptr, -1.f, -1.f, Dp, k, st));
  SH_TRY(w.red.dot(w.alpha.ptr, w.alpha.ptr, Dp, k + P, st));
  SH_TRY(w.red.comb3_sq(w.x.ptr, w.vpos.ptr, w.zpos.ptr, -1.f, -1.f, s->per, k + 2 * P, st));
  SH_TRY(w.red.dot(w.x.ptr, w.x.ptr, s->per, k + 3 * P, st));
  SH_TRY(sh::launch_kkt_vis(op, w.sphi.ptr, w.zphi.ptr, w.vphi.ptr, w.cblk.ptr, k + 8 * P, k + 8 * P + R, st));
  SH_TRY(sh::phi_adjoint(op, w.zphi.ptr, w.t2.ptr, false, w.cblk.ptr, st));          // Phi_hat^dagger z_phi
  SH_TRY(sh_psi_adj(s->psi, w.t2.ptr, w.aAp.ptr, st));
  SH_TRY(sh_psi_adj(s->psi, w.zpos.ptr, w.ap.ptr, st));
  SH_TRY(w.red.dot(w.zpsi.ptr, w.zpsi.ptr, Dp, k + 4 * P, st));
  SH_TRY(w.red.dot(w.aAp.ptr, w.aAp.ptr, Dp, k + 5 * P, st));
  SH_TRY(w.red.dot(w.ap.ptr, w.ap.ptr, Dp, k + 6 * P, st));
  SH_TRY(w.red.comb3_sq(w.zpsi.ptr, w.aAp.ptr, w.ap.ptr, 1.f, 1.f, Dp, k + 7 * P, st));
  SH_TRY(w.red.l1w(w.alpha.ptr, s->Wp, Dp, s->s_misc + MISC_OBJ * P, st));
  std::vector<double> h(8 * P + 2 * R), o(P);
  SH_HIP(hipMemcpyAsync(h.data(), k, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  SH_HIP(hipMemcpyAsync(o.data(), s->s_misc + MISC_OBJ * P, P * sizeof(double), hipMemcpyDeviceToHost, st));
  SH_HIP(hipStreamSynchronize(st));
  prim.assign(P, 0.0);
  dual.assign(P, 0.0);
  obj = o;
  for (int p = 0; p < P; ++p) {
    double pr = h[p] + h[2 * P + p], sc = h[P + p] + h[3 * P + p];
    for (int b = op->block_off[p]; b < op->block_off[p + 1]; ++b) {
      pr += h[8 * P + b] * h[8 * P + b];
      sc += h[8 * P + R + b] * h[8 * P + R + b];
    }
    prim[p] = sc > 0 ? std::sqrt(pr / sc) : 0.0;
    const double dm = std::sqrt(std::max(h[4 * P + p], std::max(h[5 * P + p], h[6 * P + p])));
    dual[p] = dm > 0 ? std::sqrt(h[7 * P + p]) / dm : 0.0;
  }
  return SH_OK;
}

// Relative KKT residuals of the current SDMM state (after at least one iteration), per problem:
//   primal = ||(s_j - y_j)_j|| / ||(s_j)_j||   over the splits j = psi, the data blocks, positivity
//            (s_j = L_j x the split images, y_j their proximal points; zero at a fixed point),
//   dual   = ||sum_j L_j^T z_j|| / max_j ||L_j^T z_j||   (stationarity of the Lagrangian).
// The state keeps v_j = y_j - z_j (data splits: c_b (y - z - s_hat)), so s_j - y_j = s_j - v_j - z_j for
// psi and positivity and -(v / c_b + z) for the data.  Also the objective ||W Psi^dagger x||_1 with the
// current weights.  Synchronises.
sh_status sdmm_kkt(sh_sdmm s, std::vector<double>& prim, std::vector<double>& dual, std::vector<double>& obj,
                   hipStream_t st) {
  sh_op op = s->op;
  Work& w = s->w;
  const int P = s->P, R = s->R;
  double* k = w.kkt.ptr;
  if (s->synth) return sdmm_kkt_synthesis(s, prim, dual, obj, st);
  SH_TRY(w.red.comb3_sq(w.spsi.ptr, w.vpsi.ptr, w.zpsi.ptr, -1.f, -1.f, s->Dper, k, st));
  SH_TRY(w.red.dot(w.spsi.ptr, w.spsi.ptr, s->Dper, k + P, st));
  SH_TRY(w.red.comb3_sq(w.x.ptr, w.vpos.ptr, w.zpos.ptr, -1.f, -1.f, s->per, k + 2 * P, st));
  SH_TRY(w.red.dot(w.x.ptr, w.x.ptr, s->per, k + 3 * P, st));
  if (s->stoch) {   // split images of every block at x_n; v_phi = c (y - z)
    SH_TRY(sh::phi_forward(op, w.x.ptr, w.vtmp.ptr, false, nullptr, st));
    SH_TRY(sh::launch_kkt_vis(op, w.vtmp.ptr, w.zphi.ptr, w.vphi.ptr, w.cblk.ptr, k + 8 * P, k + 8 * P + R, st, false));
  } else {
    SH_TRY(sh::launch_kkt_vis(op, w.sphi.ptr, w.zphi.ptr, w.vphi.ptr, w.cblk.ptr, k + 8 * P, k + 8 * P + R, st));
  }
  SH_TRY(sh_psi_fwd(s->psi, w.zpsi.ptr, w.t1.ptr, st));                              // Psi z_psi
  SH_TRY(sh::phi_adjoint(op, w.zphi.ptr, w.t2.ptr, false, w.cblk.ptr, st));          // Phi_hat^dagger z_phi
  SH_TRY(w.red.dot(w.t1.ptr, w.t1.ptr, s->per, k + 4 * P, st));
  SH_TRY(w.red.dot(w.t2.ptr, w.t2.ptr, s->per, k + 5 * P, st));
  SH_TRY(w.red.dot(w.zpos.ptr, w.zpos.ptr, s->per, k + 6 * P, st));
  SH_TRY(w.red.comb3_sq(w.t1.ptr, w.t2.ptr, w.zpos.ptr, 1.f, 1.f, s->per, k + 7 * P, st));
  SH_TRY(w.red.l1w(w.spsi.ptr, s->Wp, s->Dper, s->s_misc + MISC_OBJ * P, st));
  std::vector<double> h(8 * P + 2 * R), o(P);
  SH_HIP(hipMemcpyAsync(h.data(), k, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  SH_HIP(hipMemcpyAsync(o.data(), s->s_misc + MISC_OBJ * P, P * sizeof(double), hipMemcpyDeviceToHost, st));
  SH_HIP(hipStreamSynchronize(st));
  prim.assign(P, 0.0);
  dual.assign(P, 0.0);
  obj = o;
  for (int p = 0; p < P; ++p) {
    double pr = h[p] + h[2 * P + p], sc = h[P + p] + h[3 * P + p];
    for (int b = op->block_off[p]; b < op->block_off[p + 1]; ++b) {
      pr += h[8 * P + b] * h[8 * P + b];
      sc += h[8 * P + R + b] * h[8 * P + R + b];
    }
    prim[p] = sc > 0 ? std::sqrt(pr / sc) : 0.0;
    const double dm = std::sqrt(std::max(h[4 * P + p], std::max(h[5 * P + p], h[6 * P + p])));
    dual[p] = dm > 0 ? std::sqrt(h[7 * P + p]) / dm : 0.0;
  }
  return SH_OK;
}

sh_status sdmm_validate(sh_op op, sh_psi psi, const float* y, const double* eps, const sh_sdmm_params* prm) {
  SH_REQUIRE(op && psi && y && eps && prm, "NULL argument");
  SH_REQUIRE(psi_side(psi) == op->n, "psi and op image sides differ");
  SH_REQUIRE(psi_batch(psi) == op->P, "psi batch (%d) must equal the number of problems of op (%d)", psi_batch(psi),
             op->P);
  SH_REQUIRE(prm->max_iter >= 1 && prm->cg_iters >= 1 && prm->cg_iters <= 64 && prm->passes >= 1 &&
                 prm->check_every >= 1,
             "max_iter, passes, check_every >= 1 and cg_iters in [1, 64] required");
  SH_REQUIRE(prm->tol_rel >= 0 && prm->eps_slack >= 0 && prm->rw_beta > 0 && std::isfinite(prm->rw_beta),
             "tol_rel, eps_slack >= 0 and rw_beta > 0 required");
  SH_REQUIRE(prm->tol_dual >= 0 && std::isfinite(prm->tol_dual), "tol_dual must be finite and >= 0");
  SH_REQUIRE(prm->graph == 0 || prm->graph == 1, "graph must be 0 or 1");
  SH_REQUIRE(prm->w_from_x0 == 0 || prm->w_from_x0 == 1, "w_from_x0 must be 0 or 1");
  SH_REQUIRE(prm->z_from_x0 == 0 || prm->z_from_x0 == 1, "z_from_x0 must be 0 or 1");
  SH_REQUIRE(prm->block_fraction > 0 && prm->block_fraction <= 1, "block_fraction must be in (0, 1]");
  SH_REQUIRE(prm->block_fraction == 1 || (prm->toeplitz == 1 && prm->z_from_x0 == 0),
             "block-subset iterations (block_fraction < 1) need toeplitz = 1 and z_from_x0 = 0");
  SH_REQUIRE(prm->synthesis == 0 || prm->synthesis == 1, "synthesis must be 0 or 1");
  SH_REQUIRE(prm->synthesis == 0 || (prm->toeplitz == 1 && prm->z_from_x0 == 0 && prm->block_fraction == 1),
             "the synthesis prior needs toeplitz = 1, z_from_x0 = 0 and block_fraction = 1");
  SH_REQUIRE(prm->toeplitz == 0 || prm->toeplitz == 1, "toeplitz must be 0 or 1");
  SH_REQUIRE(prm->block_norm == 0 || prm->block_norm == 1, "block_norm must be 0 or 1");
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

}  // extern "C"

namespace {

size_t al(size_t b) { return sh::Arena::round(b); }

// Device bytes of a solver session (every allocation of its set-up, in the arena's stack order): the
// session's arrays, then the largest of the set-up's passing temporaries (the finiteness check's reducer,
// the block-weight counters, the Toeplitz build, the power iteration, the spectrum rescaling).
size_t sdmm_ws_bytes(sh_op op, int q, const sh_sdmm_params* prm) {
  const size_t P = op->P, per = size_t(op->n) * op->n, N = per * P, D = size_t(q) * per * P, M = op->M, R = op->R;
  const size_t K = op->K, KK = K * K, n = op->n, kcg = prm->cg_iters;
  const size_t rb = 512 / P > 1 ? 512 / P : 1;
  size_t pers = 9 * al(4 * N) + 4 * al(4 * D) + 5 * al(8 * M) + al(8 * (2 * kcg + 1 + MISC_N) * P) + 3 * al(8 * R) +
                al(8 * P) + al(8 * (8 * P + 2 * R)) + al(4 * R) + al(4 * P) + al(8 * 2 * P * rb) + al(8 * P * rb);
  if (prm->synthesis) pers += 5 * al(4 * D);
  if (prm->block_fraction < 1) pers += al(4 * R) + al(8) + al(4 * N);
  if (prm->toeplitz) pers += al(4 * P * KK) + al(8 * P * n * K);
  size_t tmp = al(8 * 2 * 512) + al(8 * 512);   // the finiteness check's one-segment reducer
  if (prm->block_norm) {
    const size_t G = std::max<size_t>(1, std::min<size_t>(R, (size_t(1) << 26) / KK));
    tmp = std::max(tmp, al(4 * G * KK) + al(4 * R));
  }
  if (prm->toeplitz)
    tmp = std::max(tmp, (prm->block_norm ? al(4 * R) : 0) + al(8 * M) + al(4 * P * n * n) + 2 * al(8 * P * KK) +
                            al(4 * P));
  if (!(prm->nu > 0))
    tmp = std::max(tmp, 2 * al(4 * N) + al(8 * M) + al(8 * 3 * P) + al(8 * 2 * P * rb) + al(8 * P * rb));
  return pers + tmp;
}

sh_status sdmm_create(sh_op op, sh_psi psi, const float* y, const double* eps, const float* W, const float* x0,
                      const sh_sdmm_params* params, void* workspace, size_t ws_bytes, sh_sdmm* out, void* stream) {
  SH_REQUIRE(out, "out is NULL");
  *out = nullptr;
  SH_TRY(sdmm_validate(op, psi, y, eps, params));
  SH_REQUIRE(!params->w_from_x0 || (x0 && !W), "w_from_x0 needs x0 and no W");
  SH_REQUIRE(!params->z_from_x0 || x0, "z_from_x0 needs x0");
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
  s->P = op->P;
  s->per = int64_t(op->n) * op->n;
  s->Dper = int64_t(q) * s->per;
  s->N = s->per * s->P;
  s->M = op->M;
  s->D = s->Dper * s->P;
  s->R = op->R;
  s->kcg = params->cg_iters;
  s->stoch = params->block_fraction < 1.0;
  s->synth = params->synthesis != 0;
  sh_status st;
  {
    s->arena.base = static_cast<char*>(workspace);
    s->arena.size = ws_bytes;
    sh::ArenaScope scope(workspace ? &s->arena : nullptr);
    st = sdmm_setup(s, y, eps, W, x0, (hipStream_t)stream);
  }
  if (st == SH_OK) st = hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? SH_OK : SH_EDEVICE;
  if (st == SH_OK && (hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) != hipSuccess ||
                      hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming) != hipSuccess ||
                      hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming) != hipSuccess)) {
    sh::set_error("creating the session's second stream failed");
    st = SH_EDEVICE;
  }
  if (st != SH_OK) {
    delete s;
    return st;
  }
  *out = s;
  return SH_OK;
}

// Checkpoint of a session: the state one iteration carries to the next, in this order: x, v_psi, z_psi,
// v_phi, z_phi, v_+, z_+, the data images Phi_hat x (kept per block by block-subset iterations), the block
// residuals, the weights W, then alpha (synthesis prior) and the running image Phi_hat^T v_phi and the
// iteration counter (block-subset iterations).  The header records the sizes and options it was taken with.
struct StateHeader {
  uint64_t magic;
  int64_t N, M, D, R, P;
  int32_t stoch, synth, iters_total, version;
};
constexpr uint64_t kStateMagic = 0x31545053414d4453ull;   // "SDMASPT1"

struct Part {
  void* ptr;
  size_t bytes;
};

template <typename T>
Part part(sh::DevBuf<T>& b) { return Part{b.ptr, b.count * sizeof(T)}; }

std::vector<Part> state_parts(sh_sdmm s) {
  Work& w = s->w;
  std::vector<Part> v = {part(w.x),    part(w.vpsi), part(w.zpsi), part(w.vphi),  part(w.zphi),
                         part(w.vpos), part(w.zpos), part(w.sphi), part(w.resid), part(w.W)};
  if (s->synth) v.push_back(part(w.alpha));
  if (s->stoch) {
    v.push_back(part(w.bphi));
    v.push_back(part(w.ctr));
  }
  return v;
}

StateHeader state_header(sh_sdmm s) {
  return StateHeader{kStateMagic, s->N, s->M, s->D, s->R, s->P, s->stoch ? 1 : 0, s->synth ? 1 : 0, s->iters_total, 1};
}

size_t state_bytes(sh_sdmm s) {
  size_t n = sizeof(StateHeader);
  for (const Part& q : state_parts(s)) n += q.bytes;
  return n;
}

sh_status check_ws(sh_op op, sh_psi psi, const sh_sdmm_params* params, void* workspace, size_t bytes) {
  SH_REQUIRE(op && psi && params && workspace, "NULL argument");
  SH_REQUIRE(reinterpret_cast<uintptr_t>(workspace) % sh::Arena::kAlign == 0, "workspace must be %zu-byte aligned",
             sh::Arena::kAlign);
  int32_t q = 0;
  sh_psi_planes(psi, &q);
  const size_t need = sdmm_ws_bytes(op, q, params);
  SH_REQUIRE(bytes >= need, "workspace of %zu bytes is smaller than the %zu needed", bytes, need);
  return SH_OK;
}

}  // namespace

extern "C" {

sh_status sh_workspace_bytes(sh_op op, sh_psi psi, const sh_sdmm_params* params, size_t* bytes) {
  SH_REQUIRE(op && psi && params && bytes, "NULL argument");
  int32_t q = 0;
  sh_psi_planes(psi, &q);
  *bytes = sdmm_ws_bytes(op, q, params);
  return SH_OK;
}

sh_status sh_sdmm_create(sh_op op, sh_psi psi, const float* y, const double* eps, const float* W, const float* x0,
                         const sh_sdmm_params* params, sh_sdmm* out, void* stream) {
  return sdmm_create(op, psi, y, eps, W, x0, params, nullptr, 0, out, stream);
}

sh_status sh_sdmm_create_ws(sh_op op, sh_psi psi, const float* y, const double* eps, const float* W, const float* x0,
                            const sh_sdmm_params* params, void* workspace, size_t bytes, sh_sdmm* out, void* stream) {
  SH_REQUIRE(out, "out is NULL");
  *out = nullptr;
  SH_TRY(check_ws(op, psi, params, workspace, bytes));
  return sdmm_create(op, psi, y, eps, W, x0, params, workspace, bytes, out, stream);
}

sh_status sh_sdmm_iterate(sh_sdmm s, int32_t iters, void* stream) {
  SH_REQUIRE(s && iters >= 0, "invalid argument");
  return sdmm_run(s, iters, (hipStream_t)stream);
}

sh_status sh_sdmm_result(sh_sdmm s, float* x_out, double* block_resid, double* rel_change, void* stream) {
  SH_REQUIRE(s, "NULL session");
  hipStream_t st = (hipStream_t)stream;
  if (x_out) SH_HIP(hipMemcpyAsync(x_out, s->w.x.ptr, s->N * sizeof(float), hipMemcpyDeviceToDevice, st));
  std::vector<double> rel, hres;
  SH_TRY(sdmm_read(s, rel, hres, st));
  if (block_resid)
    for (int i = 0; i < s->R; ++i) block_resid[i] = hres[i] / s->cb[i];
  if (rel_change)
    for (int p = 0; p < s->P; ++p) rel_change[p] = rel[p];
  return SH_OK;
}

sh_status sh_sdmm_kkt(sh_sdmm s, double* kkt_primal, double* kkt_dual, double* objective, void* stream) {
  SH_REQUIRE(s, "NULL session");
  SH_REQUIRE(s->iters_total > 0, "the session has not iterated yet");
  std::vector<double> pr, du, ob;
  SH_TRY(sdmm_kkt(s, pr, du, ob, (hipStream_t)stream));
  for (int p = 0; p < s->P; ++p) {
    if (kkt_primal) kkt_primal[p] = pr[p];
    if (kkt_dual) kkt_dual[p] = du[p];
    if (objective) objective[p] = ob[p];
  }
  return SH_OK;
}

sh_status sh_sdmm_state_bytes(sh_sdmm s, size_t* bytes) {
  SH_REQUIRE(s && bytes, "NULL argument");
  *bytes = state_bytes(s);
  return SH_OK;
}

sh_status sh_sdmm_state_export(sh_sdmm s, void* host, size_t bytes, void* stream) {
  SH_REQUIRE(s && host, "NULL argument");
  const size_t need = state_bytes(s);
  SH_REQUIRE(bytes >= need, "state buffer of %zu bytes is smaller than the %zu needed", bytes, need);
  hipStream_t st = (hipStream_t)stream;
  const StateHeader hd = state_header(s);
  char* p = static_cast<char*>(host);
  std::memcpy(p, &hd, sizeof hd);
  size_t off = sizeof hd;
  for (const Part& q : state_parts(s)) {
    SH_HIP(hipMemcpyAsync(p + off, q.ptr, q.bytes, hipMemcpyDeviceToHost, st));
    off += q.bytes;
  }
  SH_HIP(hipStreamSynchronize(st));
  return SH_OK;
}

sh_status sh_sdmm_state_import(sh_sdmm s, const void* host, size_t bytes, void* stream) {
  SH_REQUIRE(s && host, "NULL argument");
  const size_t need = state_bytes(s);
  SH_REQUIRE(bytes == need, "state of %zu bytes where this session takes %zu", bytes, need);
  StateHeader hd;
  std::memcpy(&hd, host, sizeof hd);
  const StateHeader mine = state_header(s);
  SH_REQUIRE(hd.magic == kStateMagic && hd.version == mine.version, "not a session state");
  SH_REQUIRE(hd.N == mine.N && hd.M == mine.M && hd.D == mine.D && hd.R == mine.R && hd.P == mine.P &&
                 hd.stoch == mine.stoch && hd.synth == mine.synth,
             "state taken from a session of other sizes or options");
  SH_REQUIRE(hd.iters_total >= 0, "invalid iteration count in the state");
  hipStream_t st = (hipStream_t)stream;
  const char* p = static_cast<const char*>(host);
  size_t off = sizeof hd;
  for (const Part& q : state_parts(s)) {
    SH_HIP(hipMemcpyAsync(q.ptr, p + off, q.bytes, hipMemcpyHostToDevice, st));
    off += q.bytes;
  }
  s->iters_total = hd.iters_total;
  if (s->ring_rows > 0) {   // the metrics ring starts again, numbered from the imported iteration count
    const unsigned long long zero = 0;
    SH_HIP(hipMemcpyAsync(s->ring_ctr.ptr, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
    s->ring_base = s->iters_total;
    s->ring_next = 0;
  }
  SH_HIP(hipStreamSynchronize(st));
  return SH_OK;
}

sh_status sh_sdmm_metrics_enable(sh_sdmm s, int32_t rows, int32_t* row_width) {
  SH_REQUIRE(s != nullptr, "session is NULL");
  SH_REQUIRE(rows >= 0 && rows <= (1 << 20), "rows must be in [0, 2^20], got %d", rows);
  SH_HIP(hipDeviceSynchronize());   // no enqueued iteration may still write the old ring
  if (s->gexec) {                   // the captured iteration carries the ring (or its absence): capture again
    SH_HIP(hipGraphExecDestroy(s->gexec));
    s->gexec = nullptr;
  }
  s->ring.release();
  s->ring_ctr.release();
  s->ring_rows = 0;
  if (row_width) *row_width = 2 * s->P + s->R;
  if (rows == 0) return SH_OK;
  SH_TRY(s->ring.alloc((size_t)rows * (size_t)(2 * s->P + s->R)));
  const unsigned long long zero = 0;
  SH_TRY(s->ring_ctr.upload(&zero, 1));
  s->ring_rows = rows;
  s->ring_base = s->iters_total;
  s->ring_next = 0;
  return SH_OK;
}

sh_status sh_sdmm_metrics_read(sh_sdmm s, double* host, int32_t max_rows, int32_t* rows_out, int64_t* first_iter,
                               void* stream) {
  SH_REQUIRE(s != nullptr && rows_out != nullptr, "NULL argument");
  SH_REQUIRE(s->ring_rows > 0, "the metrics ring is off (sh_sdmm_metrics_enable)");
  SH_REQUIRE(max_rows >= 0 && (host != nullptr || max_rows == 0), "max_rows must be >= 0 with a host buffer");
  hipStream_t st = (hipStream_t)stream;
  unsigned long long c = 0;
  SH_HIP(hipMemcpyAsync(&c, s->ring_ctr.ptr, sizeof(c), hipMemcpyDeviceToHost, st));
  SH_HIP(hipStreamSynchronize(st));
  const unsigned long long G = (unsigned long long)s->ring_rows, W = (unsigned long long)(2 * s->P + s->R);
  const unsigned long long lo = std::max(s->ring_next, c > G ? c - G : 0ull);   // older rows were overwritten
  const unsigned long long n = std::min<unsigned long long>(c - lo, (unsigned long long)max_rows);
  for (unsigned long long k = 0; k < n;) {   // at most two contiguous pieces of the ring
    const unsigned long long slot = (lo + k) % G, len = std::min(n - k, G - slot);
    SH_HIP(hipMemcpyAsync(host + k * W, s->ring.ptr + slot * W, len * W * sizeof(double), hipMemcpyDeviceToHost, st));
    k += len;
  }
  SH_HIP(hipStreamSynchronize(st));
  s->ring_next = lo + n;
  *rows_out = (int32_t)n;
  if (first_iter) *first_iter = (int64_t)s->ring_base + (int64_t)lo + 1;
  return SH_OK;
}

sh_status sh_sdmm_destroy(sh_sdmm s) {
  delete s;
  return SH_OK;
}

}  // extern "C"

namespace {

sh_status sdmm_solve(sh_op op, sh_psi psi, const float* y, const double* eps, const float* W0, const float* x0,
                     const sh_sdmm_params* prm, float* x_out, float* W_out, double* block_resid, sh_sdmm_info* info,
                     void* workspace, size_t ws_bytes, void* stream) {
  const auto t_start = std::chrono::steady_clock::now();
  SH_REQUIRE(x_out, "x_out is NULL");
  sh_sdmm s = nullptr;
  SH_TRY(sdmm_create(op, psi, y, eps, W0, x0, prm, workspace, ws_bytes, &s, stream));
  std::unique_ptr<sh_sdmm_s> guard(s);
  hipStream_t st = (hipStream_t)stream;
  const int P = s->P;
  const int64_t per = s->per;
  std::vector<double> rel(P, INFINITY), hres;
  // Per problem: its pass, iterations in that pass, iterations of each finished pass, and whether it
  // is done (its last pass ended).  With a stopping test every problem of a batch moves through its
  // passes on its own: when its test holds (or its pass reaches max_iter) it is reweighted and starts
  // its next pass at once, and after its last pass its image, residuals, relative change and KKT
  // residuals are taken, while the batch iterates on for the others.  So a batched solve returns what
  // each problem would give alone (when max_iter is a multiple of check_every).  Without a stopping
  // test all passes have max_iter iterations and every problem reweights together.
  std::vector<int> pass(P, 0), itp(P, 0), done(P, 0), conv(P, 0);
  std::vector<std::vector<int>> pass_it(P);
  std::vector<double> rel_out(P, INFINITY), res_out(s->R, 0.0), kp_out(P, 0.0), kd_out(P, 0.0);
  auto take = [&](int p, std::vector<double>& kp, std::vector<double>& kd) -> sh_status {
    SH_HIP(hipMemcpyAsync(x_out + p * per, s->w.x.ptr + p * per, per * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (s->synth)
      SH_HIP(hipMemcpyAsync(s->w.alpha_out.ptr + p * s->Dper, s->w.alpha.ptr + p * s->Dper, s->Dper * sizeof(float),
                            hipMemcpyDeviceToDevice, st));
    rel_out[p] = rel[p];
    for (int i = op->block_off[p]; i < op->block_off[p + 1]; ++i) res_out[i] = hres[i] / s->cb[i];
    kp_out[p] = kp[p];
    kd_out[p] = kd[p];
    done[p] = 1;
    return SH_OK;
  };
  if (prm->tol_rel > 0) {
    for (;;) {
      int chunk = prm->check_every;
      for (int p = 0; p < P; ++p)
        if (!done[p]) chunk = std::min(chunk, prm->max_iter - itp[p]);
      SH_TRY(sdmm_run(s, chunk, st));
      for (int p = 0; p < P; ++p)
        if (!done[p]) itp[p] += chunk;
      SH_TRY(sdmm_read(s, rel, hres, st));
      // relative change and feasibility, then (option tol_dual) the relative dual residual, evaluated only
      // when some problem passed the first two
      std::vector<char> ok(P, 0);
      bool any = false;
      for (int p = 0; p < P; ++p) {
        if (done[p]) continue;
        bool k = rel[p] <= prm->tol_rel;
        for (int i = op->block_off[p]; k && i < op->block_off[p + 1]; ++i)
          k = hres[i] <= s->eh[i] * (1.0 + prm->eps_slack);
        ok[p] = k;
        any = any || k;
      }
      std::vector<double> kp, kd, ko;
      bool have_kkt = false;
      if (any && prm->tol_dual > 0) {
        SH_TRY(sdmm_kkt(s, kp, kd, ko, st));
        have_kkt = true;
        for (int p = 0; p < P; ++p) ok[p] = ok[p] && kd[p] <= prm->tol_dual;
      }
      std::vector<char> next(P, 0);   // problems whose pass ended and that go on to another pass
      bool finishing = false;
      for (int p = 0; p < P; ++p) {
        if (done[p] || !(ok[p] || itp[p] >= prm->max_iter)) continue;
        pass_it[p].push_back(itp[p]);
        if (pass[p] + 1 == prm->passes) {
          conv[p] = ok[p];
          finishing = true;
        } else {
          next[p] = 1;
          ++pass[p];
          itp[p] = 0;
        }
      }
      if (finishing) {
        if (!have_kkt) SH_TRY(sdmm_kkt(s, kp, kd, ko, st));
        for (int p = 0; p < P; ++p)
          if (!done[p] && (int)pass_it[p].size() == prm->passes) SH_TRY(take(p, kp, kd));
      }
      bool any_next = false;
      for (int p = 0; p < P; ++p) any_next = any_next || next[p];
      if (any_next) SH_TRY(sdmm_reweight(s, s->w.W.ptr, st, &next));   // from Psi^dagger x_n (in spsi)
      bool all = true;
      for (int p = 0; p < P; ++p) all = all && done[p];
      if (all) break;
    }
  } else {
    for (int t = 0; t < prm->passes; ++t) {
      SH_TRY(sdmm_run(s, prm->max_iter, st));
      for (int p = 0; p < P; ++p) pass_it[p].push_back(prm->max_iter);
      if (t + 1 < prm->passes) SH_TRY(sdmm_reweight(s, s->w.W.ptr, st));
    }
    SH_TRY(sdmm_read(s, rel, hres, st));
    std::vector<double> kp, kd, ko;
    SH_TRY(sdmm_kkt(s, kp, kd, ko, st));
    for (int p = 0; p < P; ++p) SH_TRY(take(p, kp, kd));
  }
  // objective with the last pass's weights and W_out, both from the returned images' coefficients:
  // Psi^dagger x (analysis) or the alpha taken with x (synthesis)
  const float* coeffs = s->w.spsi.ptr;
  if (s->synth)
    coeffs = s->w.alpha_out.ptr;
  else
    SH_TRY(sh_psi_adj(s->psi, x_out, s->w.spsi.ptr, st));
  SH_TRY(s->w.red.l1w(coeffs, s->Wp, s->Dper, s->s_misc + MISC_OBJ * P, st));
  if (W_out) SH_TRY(sdmm_reweight(s, W_out, st, nullptr, coeffs));
  std::vector<double> obj(P);
  SH_HIP(hipMemcpyAsync(obj.data(), s->s_misc + MISC_OBJ * P, P * sizeof(double), hipMemcpyDeviceToHost, st));
  SH_HIP(hipStreamSynchronize(st));
  if (block_resid) std::copy(res_out.begin(), res_out.end(), block_resid);
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (info)
    for (int p = 0; p < P; ++p) {
      sh_sdmm_info& inf = info[p];
      inf = sh_sdmm_info{};
      for (int v : pass_it[p]) inf.iters_total += v;
      inf.passes_done = (int)pass_it[p].size();
      inf.converged = prm->tol_rel > 0 ? conv[p] : 0;
      inf.iters_last = pass_it[p].empty() ? 0 : pass_it[p].back();
      inf.rel_change = rel_out[p];
      inf.objective = obj[p];
      inf.gamma = s->gamma[p];
      inf.nu = s->nu[p];
      inf.delta = s->delta[p];
      inf.seconds = secs;
      inf.kkt_primal = kp_out[p];
      inf.kkt_dual = kd_out[p];
      for (int t = 0; t < (int)pass_it[p].size() && t < SH_PASS_RECORD; ++t) inf.pass_iters[t] = pass_it[p][t];
    }
  return SH_OK;
}

}  // namespace

extern "C" {

sh_status sh_sdmm_solve(sh_op op, sh_psi psi, const float* y, const double* eps, const float* W0, const float* x0,
                        const sh_sdmm_params* prm, float* x_out, float* W_out, double* block_resid,
                        sh_sdmm_info* info, void* stream) {
  return sdmm_solve(op, psi, y, eps, W0, x0, prm, x_out, W_out, block_resid, info, nullptr, 0, stream);
}

sh_status sh_sdmm_solve_ws(sh_op op, sh_psi psi, const float* y, const double* eps, const float* W0, const float* x0,
                           const sh_sdmm_params* prm, float* x_out, float* W_out, double* block_resid,
                           sh_sdmm_info* info, void* workspace, size_t bytes, void* stream) {
  SH_TRY(check_ws(op, psi, prm, workspace, bytes));
  return sdmm_solve(op, psi, y, eps, W0, x0, prm, x_out, W_out, block_resid, info, workspace, bytes, stream);
}

}  // extern "C"
