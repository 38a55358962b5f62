// Internal launchers of the proximal steps and float64 reductions (prox.hip).
#pragma once

#include "op.hpp"

namespace sh {

// Two-stage deterministic float64 reductions; results land in device memory.
struct Reducer {
  DevBuf<double> part;
  sh_status init();
  sh_status dot(const float* a, const float* b, int64_t N, double* out, hipStream_t st);
  sh_status std_dev(const float* a, int64_t N, double* sum_out, double* var_out, hipStream_t st);  // var_out = sum (a-mean)^2
  sh_status maxabs(const float* a, int64_t N, double* out, hipStream_t st);
  sh_status l1w(const float* c, const float* W, int64_t N, double* out, hipStream_t st);
};

sh_status launch_prox_l1(int64_t D, const float* s, float* z, const float* W, float gamma, float* v, hipStream_t st);
sh_status launch_prox_pos(int64_t N, const float* s, float* z, float* v, hipStream_t st);
sh_status launch_prox_ball(sh_op op, const float2* s, float2* z, const float2* yhat, const double* eps, double* rho,
                           double* resid, float2* v, bool sub_s, hipStream_t st);
sh_status launch_reweight(int64_t D, const float* c, double delta, float* W, hipStream_t st);

}  // namespace sh
