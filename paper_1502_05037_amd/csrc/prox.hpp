// Internal launchers of the proximal steps and float64 reductions (prox.hip).
#pragma once

#include "op.hpp"

namespace sh {

// Two-stage deterministic float64 reductions over P equal segments of length `per` (segment p is
// a[p*per, (p+1)*per)); segment p's result lands in out[p] (device memory).  The tree depends only on
// (per, P), so results are reproducible bit for bit.
struct Reducer {
  DevBuf<double> part, part2;   // first-stage partials (part2: the r.r partials between cg_update and cg_dir)
  int P = 1, rb = 512;   // segments, first-stage work-groups per segment
  sh_status init(int segments = 1);
  sh_status dot(const float* a, const float* b, int64_t per, double* out, hipStream_t st);
  // sum_out[p] = sum of segment p, var_out[p] = sum of its squared deviations from its mean
  sh_status std_dev(const float* a, int64_t per, double* sum_out, double* var_out, hipStream_t st);
  sh_status maxabs(const float* a, int64_t per, double* out, hipStream_t st);
  sh_status l1w(const float* c, const float* W, int64_t per, double* out, hipStream_t st);
  // out[p] = sum over segment p of (a + fb b + fc c)^2 (b, c may be NULL)
  sh_status comb3_sq(const float* a, const float* b, const float* c, float fb, float fc, int64_t per, double* out,
                     hipStream_t st);
  // Conjugate-gradient steps fused with the reductions around them (same trees as dot).  A step is cg_ap,
  // cg_update, then (unless it is the last) cg_dir; the final sum of a dot product is taken by every
  // work-group of the kernel that consumes it, not by a launch of its own:
  //   cg_init:   r = a + b + c - xc x (c may be NULL), p = r, xprev = x;  rs_out = r.r
  //   cg_ap:     Ap = pc p + Ap;  partials of p.Ap
  //   cg_update: pap_out = p.Ap, alpha = rs / pap, x += alpha p, r -= alpha Ap;  partials of r.r
  //   cg_dir:    rs_out = r.r, beta = rs_out / rs, p = r + beta p
  //   change:    out2[0..P) = ||x - xprev||^2, out2[P..2P) = ||x||^2
  sh_status cg_init(const float* a, const float* b, const float* c, const float* x, float* r, float* p, float* xprev,
                    int64_t per, double* rs_out, hipStream_t st, float xc = 2.f);
  sh_status cg_ap(const float* p, float* Ap, int64_t per, hipStream_t st, float pc = 2.f);
  sh_status cg_update(float* x, float* r, const float* p, const float* Ap, int64_t per, const double* rs,
                      double* pap_out, hipStream_t st);
  sh_status cg_dir(const float* r, float* p, int64_t per, const double* rs, double* rs_out, hipStream_t st);
  sh_status change(const float* x, const float* xprev, int64_t per, double* out2, hipStream_t st);
};

// Elementwise proximal steps over P segments of length `per`; segment p uses gamma[p] / delta[p]
// (device arrays) or, if those are NULL, the scalar.
sh_status launch_prox_l1(int64_t per, int P, const float* s, float* z, const float* W, const float* gamma_d,
                         float gamma, float* v, hipStream_t st);
sh_status launch_prox_pos(int64_t N, const float* s, float* z, float* v, hipStream_t st);
// cblk: per-block weights c_b (device R floats) or NULL (1): the split uses c_b s (s = Phi x unweighted)
// and v is returned multiplied by c_b, ready for the unweighted adjoint.
// Only the block norms of the ball step: rho_b = ||c_b s_b + z_b - yhat_b||, resid_b = ||c_b s_b - yhat_b||.
sh_status ball_norms_only(sh_op op, const float2* s, const float2* z, const float2* yhat, const float* cblk, double* rho,
                          double* resid, hipStream_t st);
// The same without timing events (sh_prox_ball_noalloc).
sh_status ball_kernels(sh_op op, const float2* s, float2* z, const float2* yhat, const double* eps, double* rho,
                       double* resid, float2* v, bool sub_s, const float* cblk, hipStream_t st);
sh_status launch_prox_ball(sh_op op, const float2* s, float2* z, const float2* yhat, const double* eps, double* rho,
                           double* resid, float2* v, bool sub_s, const float* cblk, hipStream_t st);
// Primal residual of the data splits per block: prim_b[b] = ||s_hat_b - y_b||, from v = c (y - z - s_hat)
// (sub_s) or v = c (y - z), and scale_b[b] = ||c_b s_b|| (device R doubles each).
sh_status launch_kkt_vis(sh_op op, const float2* s, const float2* z, const float2* v, const float* cblk, double* prim_b,
                         double* scale_b, hipStream_t st, bool sub_s = true);
// Block-subset ball step: only blocks with bmask[b] != 0 are projected; v = c_b (y - z) and dv = v_new - v_old
// for those blocks (the other blocks' z, v and dv are left as they are).  resid/rho of unselected blocks are
// stale.
sh_status launch_prox_ball_subset(sh_op op, const float2* s, float2* z, const float2* yhat, const double* eps,
                                 double* rho, double* resid, float2* v, float2* dv, const float* cblk,
                                 const int32_t* bmask, hipStream_t st);
sh_status launch_reweight(int64_t per, int P, const float* c, const double* delta_d, double delta, float* W,
                          hipStream_t st);

}  // namespace sh
