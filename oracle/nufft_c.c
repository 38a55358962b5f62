/*
 * Interpolation step G of the FP64 oracle NUFFT, in plain C with OpenMP (test
 * infrastructure only: it checks the HIP library and shares no code with it).
 *
 * The measurement operator of the paper's model y = Phi x + n is realised as
 * Phi = G F Z S; the Python side (oracle/measurement.py) does S, Z and F with
 * numpy/scipy FFTs and calls these two loops for G and its adjoint G^H, which
 * are too slow in numpy for millions of visibilities.  Definitions (the same as
 * the numpy oracle's):
 *   kappa = u K / (2 pi), taps j = floor(kappa) - J/2 + 1 + t, t = 0..J-1, mod K,
 *   psi(s) = I0(beta sqrt(1 - (2 s / J)^2)) / I0(beta) for |s| <= J/2, else 0,
 *   (G X)_m = sum_{t1, t2} psi(kappa_m1 - j1) psi(kappa_m2 - j2) X[j1 mod K, j2 mod K],
 *   (G^H v)[a, b] = sum_m psi(kappa_m1 - j1) psi(kappa_m2 - j2) v_m over the taps (j1, j2) = (a, b) mod K.
 * The weights are computed once per operator (oracle_taps) and reused by both loops, which visit
 * the visibilities in the order the caller gives (the Python side passes them sorted by grid cell, so
 * that neighbouring visibilities touch neighbouring grid rows; the order only changes the rounding of
 * the adjoint's sums).
 * I0 is summed from its power series sum_k ((x/2)^2)^k / (k!)^2, which for
 * 0 <= x <= 40 reaches full float64 accuracy in under 80 terms (all terms are
 * positive, so there is no cancellation).
 * Complex arrays are interleaved (re, im) float64 pairs; X and the grid are
 * K x K row-major (first index from u, second from v).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <sys/mman.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* 1 / k^2 for the Bessel series */
static double inv_sq[200];
static void init_inv_sq(void) {
  if (inv_sq[1] != 0.0) return;
  for (int k = 1; k < 200; ++k) inv_sq[k] = 1.0 / ((double)k * (double)k);
}

double oracle_bessel_i0(double x) {
  init_inv_sq();
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 200; ++k) {
    term *= q * inv_sq[k];
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

/* Kaiser-Bessel window at offset s (a single value, for testing the series against a library). */
double oracle_kb(double s, int J, double beta) {
  init_inv_sq();
  const double a = 1.0 - (2.0 * s / J) * (2.0 * s / J);
  if (a < 0.0) return 0.0;
  return oracle_bessel_i0(beta * sqrt(a)) / oracle_bessel_i0(beta);
}

/* Taps of every visibility: j0[2m + a] = floor(kappa) - J/2 + 1 (not yet reduced mod K) and
 * w[(2m + a) J + t] = psi(kappa - j0 - t) along axis a (0: u, 1: v).  uv: M x 2 float64 (radians per
 * pixel). */
void oracle_taps(int64_t M, const double* uv, int K, int J, double beta, int64_t* j0, double* w, int nthreads) {
  init_inv_sq();
  const double i0b = oracle_bessel_i0(beta);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t i = 0; i < 2 * M; ++i) {
    const double kappa = uv[i] * ((double)K / (2.0 * M_PI));
    const int64_t base = (int64_t)floor(kappa) - J / 2 + 1;
    j0[i] = base;
    for (int t = 0; t < J; ++t) {
      const double s = kappa - (double)(base + t);
      const double a = 1.0 - (2.0 * s / J) * (2.0 * s / J);
      w[i * J + t] = a < 0.0 ? 0.0 : oracle_bessel_i0(beta * sqrt(a)) / i0b;
    }
  }
}

/* zeroed buffer of n doubles on 2 MiB pages where the kernel allows it (the grids are read and
 * written at random rows: small pages would cost a TLB miss per tap row) */
static double* grid_alloc(size_t n) {
  void* p = NULL;
  const size_t bytes = (n * sizeof(double) + (2u << 20) - 1) & ~(size_t)((2u << 20) - 1);
  if (posix_memalign(&p, 2u << 20, bytes) != 0) return NULL;
  (void)madvise(p, bytes, MADV_HUGEPAGE);
  memset(p, 0, bytes);
  return (double*)p;
}

static int64_t wrap(int64_t j, int64_t K) {
  const int64_t r = j % K;
  return r < 0 ? r + K : r;
}

/* out[idx[i]] = (G X) at the visibility whose taps are row i of oracle_taps' output, i < M. */
void oracle_interp_fwd(int64_t M, int K, int J, const int64_t* j0, const double* w, const int64_t* idx,
                       const double* X, double* out, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t m = 0; m < M; ++m) {
    const double* w1 = w + (2 * m) * J;
    const double* w2 = w + (2 * m + 1) * J;
    int64_t cols[32];
    for (int t2 = 0; t2 < J; ++t2) cols[t2] = wrap(j0[2 * m + 1] + t2, K);
    double re = 0.0, im = 0.0;
    for (int t1 = 0; t1 < J; ++t1) {
      const int64_t r = wrap(j0[2 * m] + t1, K);
      for (int t2 = 0; t2 < J; ++t2) {
        const int64_t c = cols[t2];
        const double ww = w1[t1] * w2[t2];
        re += ww * X[2 * (r * K + c)];
        im += ww * X[2 * (r * K + c) + 1];
      }
    }
    out[2 * idx[m]] = re;
    out[2 * idx[m] + 1] = im;
  }
}

/* grid = G^H v (overwritten): visibility idx[i] spread with the taps of row i of oracle_taps' output.
 * Each thread sums a contiguous range of rows into a private grid; the private grids are then added in
 * thread order.  Returns 0, or -1 if memory ran out. */
int oracle_interp_adj(int64_t M, int K, int J, const int64_t* j0, const double* w, const int64_t* idx,
                      const double* v, double* grid, int nthreads) {
  const int64_t KK = (int64_t)K * K;
  int T = 1;
#ifdef _OPENMP
  T = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
  double* priv = grid_alloc((size_t)T * 2 * KK);
  if (!priv) return -1;
#ifdef _OPENMP
#pragma omp parallel num_threads(T)
#endif
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    const int64_t lo = M * tid / T, hi = M * (tid + 1) / T;
    double* g = priv + (size_t)tid * 2 * KK;
    for (int64_t m = lo; m < hi; ++m) {
      const double* w1 = w + (2 * m) * J;
      const double* w2 = w + (2 * m + 1) * J;
      const double vr = v[2 * idx[m]], vi = v[2 * idx[m] + 1];
      int64_t cols[32];
      for (int t2 = 0; t2 < J; ++t2) cols[t2] = wrap(j0[2 * m + 1] + t2, K);
      for (int t1 = 0; t1 < J; ++t1) {
        const int64_t r = wrap(j0[2 * m] + t1, K);
        for (int t2 = 0; t2 < J; ++t2) {
          const int64_t c = cols[t2];
          const double ww = w1[t1] * w2[t2];
          g[2 * (r * K + c)] += ww * vr;
          g[2 * (r * K + c) + 1] += ww * vi;
        }
      }
    }
  }
  /* fixed-order sum of the private grids */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(T)
#endif
  for (int64_t i = 0; i < 2 * KK; ++i) {
    double s = 0.0;
    for (int t = 0; t < T; ++t) s += priv[(size_t)t * 2 * KK + i];
    grid[i] = s;
  }
  free(priv);
  return 0;
}
