// Autotuner of the measurement-operator plan: kernel width from an accuracy target, tiling by timing.
//
// Kernel width.  With the Kaiser-Bessel window psi and its transform psi_hat, interpolating from an
// alpha-times oversampled grid aliases the image spectrum: at image frequency xi (cycles per grid
// cell, |xi| <= 1/(2 alpha)) the replicas psi_hat(xi + l), l != 0, leak in against the main term
// psi_hat(xi).  The estimate used here is the RMS over xi of
//   E(xi) = sqrt(sum_{l != 0} psi_hat(xi + l)^2) / |psi_hat(xi)|,
// times sqrt(2) for the two axes: the relative error of Phi against the exact sum (1)'s measurement
// operator for an image of unit-variance white noise.  The tuner takes the smallest even J whose
// estimate meets the caller's target.
//
// Tiling.  For that J it builds plans with gridding tile sides {8, 16, 32} (default item cap), then,
// for the fastest tile, item caps {1024, 16384}; each candidate is timed as `reps` applications of
// Phi and Phi^dagger in internal order after one untimed application, with HIP events on the
// caller's stream.  The fastest plan is returned, and the choice is remembered for the process
// under a key of the sizes and a hash of the uv points and block offsets, so that re-planning the
// same data skips the timing.  With the environment variable SH_TUNE_CACHE naming a file, the choices
// also persist across processes: a key the process has not seen is looked up in that file, and every
// new choice is appended to it as one line "sarahip-tune-1 <key> <J> <tile> <chunk> <ms>".  The key
// starts with the library version, so that another build times again; the last valid line of a key
// wins; a line that does not parse or names a tiling the plan refuses is skipped.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "op.hpp"
#include "tables.hpp"

#define SH_TUNE_VERSION "sarahip-0.1-gfx950"

namespace {

double alias_estimate(int J, int alpha) {
  const double beta = sh::kb_beta(J, alpha);
  const int nx = 257, L = 2000;
  double acc = 0.0;
  for (int k = 0; k < nx; ++k) {
    const double xi = (double(k) / (nx - 1) - 0.5) / alpha;
    double s = 0.0;
    for (int l = 1; l <= L; ++l) {
      const double a = sh::kb_transform(xi + l, J, beta), b = sh::kb_transform(xi - l, J, beta);
      s += a * a + b * b;
    }
    const double m = sh::kb_transform(xi, J, beta);
    acc += s / (m * m);
  }
  return std::sqrt(2.0 * acc / nx);
}

struct Choice {
  int J, tile, chunk;
  double ms;
};
std::mutex g_mu;
std::map<std::string, Choice> g_cache;

uint64_t fnv(const void* p, size_t n, uint64_t h) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

std::string cache_key(const double* uv, const int64_t* M_p, int P, int n, int alpha, double acc,
                      const int64_t* offs, const int32_t* R_p) {
  int64_t M = 0, R = 0;
  for (int p = 0; p < P; ++p) {
    M += M_p[p];
    R += R_p[p];
  }
  uint64_t h = 1469598103934665603ull;
  h = fnv(M_p, P * sizeof(int64_t), h);
  h = fnv(R_p, P * sizeof(int32_t), h);
  h = fnv(offs, (R + 1) * sizeof(int64_t), h);
  h = fnv(uv, 2 * M * sizeof(double), h);
  char buf[200];
  std::snprintf(buf, sizeof(buf), "%s/%d/%d/%d/%.6e/%lld/%llx", SH_TUNE_VERSION, n, P, alpha, acc, (long long)M,
                (unsigned long long)h);
  return buf;
}

constexpr const char* kTuneTag = "sarahip-tune-1";

// The last line of the cache file for `key` with kernel width J and a tiling the planner accepts.
bool file_lookup(const std::string& key, int J, Choice* out) {
  const char* path = std::getenv("SH_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512], tag[32], k[256];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    Choice c{};
    if (std::sscanf(line, "%31s %255s %d %d %d %lf", tag, k, &c.J, &c.tile, &c.chunk, &c.ms) != 6) continue;
    if (std::strcmp(tag, kTuneTag) != 0 || key != k || c.J != J) continue;
    if ((c.tile != 8 && c.tile != 16 && c.tile != 32) || c.chunk < 64 || c.chunk > (1 << 20) || !(c.ms > 0)) continue;
    *out = c;
    found = true;
  }
  std::fclose(f);
  return found;
}

void file_append(const std::string& key, const Choice& c) {
  const char* path = std::getenv("SH_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;   // a cache that cannot be written only costs the next process a tuning
  std::fprintf(f, "%s %s %d %d %d %.6g\n", kTuneTag, key.c_str(), c.J, c.tile, c.chunk, c.ms);
  std::fclose(f);
}

__global__ void fill_ones(float* a, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) a[i] = 1.0f;
}

// Mean milliseconds of one Phi + Phi^dagger pair of `op` on `st`.
sh_status time_pair(sh_op op, float* x, float2* vis, int reps, hipStream_t st, double* ms) {
  SH_TRY(sh::phi_forward(op, x, vis, false, nullptr, st));
  SH_TRY(sh::phi_adjoint(op, vis, x, false, nullptr, st));
  hipEvent_t a, b;
  SH_HIP(hipEventCreate(&a));
  SH_HIP(hipEventCreate(&b));
  sh_status s = SH_OK;
  (void)hipEventRecord(a, st);
  for (int r = 0; r < reps && s == SH_OK; ++r) {
    s = sh::phi_forward(op, x, vis, false, nullptr, st);
    if (s == SH_OK) s = sh::phi_adjoint(op, vis, x, false, nullptr, st);
  }
  (void)hipEventRecord(b, st);
  float t = 0.f;
  if (s == SH_OK && (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&t, a, b) != hipSuccess)) {
    sh::set_error("timing the operator failed");
    s = SH_EDEVICE;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = double(t) / reps;
  return s;
}

}  // namespace

extern "C" {

sh_status sh_kb_alias_error(int32_t kernel_width, int32_t oversample, double* err_out) {
  SH_REQUIRE(err_out, "NULL argument");
  SH_REQUIRE(kernel_width >= 2 && kernel_width <= 16 && kernel_width % 2 == 0, "J must be even in [2, 16]");
  SH_REQUIRE(oversample == 2 || oversample == 4, "oversample must be 2 or 4");
  *err_out = alias_estimate(kernel_width, oversample);
  return SH_OK;
}

sh_status sh_op_autotune(const double* uv, const int64_t* M_p, int32_t P, int32_t n, int32_t oversample,
                         double accuracy, const int64_t* block_offsets, const int32_t* R_p, int32_t reps,
                         sh_tune_result* result, sh_op* out, void* stream) {
  SH_REQUIRE(out && result && uv && M_p && block_offsets && R_p, "NULL argument");
  *out = nullptr;
  SH_REQUIRE(P >= 1 && P <= 4096, "P must be in [1, 4096]");
  SH_REQUIRE(oversample == 2 || oversample == 4, "oversample must be 2 or 4");
  SH_REQUIRE(std::isfinite(accuracy) && accuracy > 0 && accuracy < 1, "accuracy must be in (0, 1)");
  SH_REQUIRE(reps >= 1 && reps <= 1000, "reps must be in [1, 1000]");
  hipStream_t st = (hipStream_t)stream;
  std::memset(result, 0, sizeof(*result));
  result->accuracy = accuracy;
  int J = 0;
  for (int j = 2; j <= 16 && !J; j += 2)
    if (alias_estimate(j, oversample) <= accuracy) J = j;
  SH_REQUIRE(J > 0, "no kernel width up to 16 reaches accuracy %g", accuracy);
  result->J = J;
  result->alias_error = alias_estimate(J, oversample);
  const std::string key = cache_key(uv, M_p, P, n, oversample, accuracy, block_offsets, R_p);
  {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      const Choice c = it->second;
      result->tile = c.tile;
      result->chunk = c.chunk;
      result->ms_pair = c.ms;
      result->cached = 1;
      return sh_op_create_batched(uv, M_p, P, n, oversample, J, block_offsets, R_p, c.tile, c.chunk, out);
    }
  }
  {
    Choice c{};
    if (file_lookup(key, J, &c) &&
        sh_op_create_batched(uv, M_p, P, n, oversample, J, block_offsets, R_p, c.tile, c.chunk, out) == SH_OK) {
      std::lock_guard<std::mutex> g(g_mu);
      g_cache[key] = c;
      result->tile = c.tile;
      result->chunk = c.chunk;
      result->ms_pair = c.ms;
      result->cached = 2;
      return SH_OK;
    }
  }
  // scratch for timing
  int64_t M = 0;
  for (int p = 0; p < P; ++p) M += M_p[p];
  const int64_t N = int64_t(P) * n * n;
  sh::DevBuf<float> x;
  sh::DevBuf<float2> vis;
  SH_TRY(x.alloc(N));
  SH_TRY(vis.alloc(M));
  hipLaunchKernelGGL(fill_ones, dim3((unsigned)sh::cdiv(N, 256)), dim3(256), 0, st, x.ptr, N);
  SH_LAUNCHED();

  sh_op best = nullptr;
  Choice bc{J, 0, 0, 1e30};
  auto consider = [&](int tile, int chunk) -> sh_status {
    sh_op op = nullptr;
    const sh_status s = sh_op_create_batched(uv, M_p, P, n, oversample, J, block_offsets, R_p, tile, chunk, &op);
    if (s == SH_EINVAL && tile != 0) return SH_OK;   // tile does not fit this grid: not a candidate
    SH_TRY(s);
    double ms = 0;
    const sh_status ts = time_pair(op, x.ptr, vis.ptr, reps, st, &ms);
    if (ts != SH_OK) {
      sh_op_destroy(op);
      return ts;
    }
    result->candidates += 1;
    if (ms < bc.ms) {
      if (best) sh_op_destroy(best);
      best = op;
      bc = Choice{J, op->T, op->chunk, ms};
    } else {
      sh_op_destroy(op);
    }
    return SH_OK;
  };
  sh_status s = SH_OK;
  for (int tile : {8, 16, 32})
    if (s == SH_OK) s = consider(tile, 0);
  if (s == SH_OK && !best) s = consider(0, 0);
  const int t_best = bc.tile;
  for (int chunk : {1024, 16384})
    if (s == SH_OK) s = consider(t_best, chunk);
  if (s != SH_OK) {
    if (best) sh_op_destroy(best);
    return s;
  }
  {
    std::lock_guard<std::mutex> g(g_mu);
    g_cache[key] = bc;
  }
  file_append(key, bc);
  result->tile = bc.tile;
  result->chunk = bc.chunk;
  result->ms_pair = bc.ms;
  *out = best;
  return SH_OK;
}

sh_status sh_tune_cache_clear(void) {
  std::lock_guard<std::mutex> g(g_mu);
  g_cache.clear();
  return SH_OK;
}

}  // extern "C"
