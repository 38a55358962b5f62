// Host-side float64 tables of the library: Kaiser-Bessel kernel (interpolation polynomials and the
// deapodisation profile), Daubechies filters, FFT twiddles.  Everything here runs once per plan.
#include "tables.hpp"

#include <cmath>
#include <complex>
#include <cstring>

namespace sh {

// Modified Bessel function of the first kind, order 0: sum_k (x^2/4)^k / (k!)^2 (all terms positive).
double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 500; ++k) {
    term *= q / (double(k) * double(k));
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return sum;
}

double kb_beta(int J, int alpha) {
  const double a = double(alpha), w = double(J);
  return M_PI * std::sqrt((w / a) * (w / a) * (a - 0.5) * (a - 0.5) - 0.8);
}

double kb_window(double t, int J, double beta) {
  const double u = 2.0 * t / J;
  const double arg = 1.0 - u * u;
  if (arg < 0.0) return 0.0;
  return bessel_i0(beta * std::sqrt(arg)) / bessel_i0(beta);
}

// Fourier transform of the window: J sinh(z)/z / I0(beta), z = sqrt(beta^2 - (pi J xi)^2);
// for pi J |xi| > beta the root is imaginary and sinh(z)/z = sin(w)/w.
double kb_transform(double xi, int J, double beta) {
  const double z2 = beta * beta - (M_PI * J * xi) * (M_PI * J * xi);
  double r;
  if (z2 > 0) {
    const double z = std::sqrt(z2);
    r = std::sinh(z) / z;
  } else if (z2 < 0) {
    const double w = std::sqrt(-z2);
    r = std::sin(w) / w;
  } else {
    r = 1.0;
  }
  return J * r / bessel_i0(beta);
}

// Per-tap interpolation polynomials.  For base cell floor(kappa) and fraction f in [0, 1), tap t
// (t = 0..J-1) sits at distance f + J/2 - 1 - t; its weight is approximated by a degree-`deg`
// polynomial in s = 2f - 1 obtained by Chebyshev interpolation and expanded to monomials.
void kb_tap_polys(int J, double beta, int deg, float* coef /* J*(deg+1), row t */) {
  const int nn = deg + 1;
  std::vector<double> node(nn), cheb(nn);
  for (int t = 0; t < J; ++t) {
    std::vector<double> val(nn);
    for (int k = 0; k < nn; ++k) {
      node[k] = std::cos(M_PI * (k + 0.5) / nn);
      const double f = 0.5 * (node[k] + 1.0);
      val[k] = kb_window(f + J / 2 - 1 - t, J, beta);
    }
    for (int j = 0; j < nn; ++j) {
      double acc = 0.0;
      for (int k = 0; k < nn; ++k) acc += val[k] * std::cos(j * M_PI * (k + 0.5) / nn);
      cheb[j] = acc * 2.0 / nn;
    }
    cheb[0] *= 0.5;
    // monomial expansion via T_{j+1} = 2 s T_j - T_{j-1}
    std::vector<double> mono(nn, 0.0), tm1(nn, 0.0), tj(nn, 0.0), tn(nn, 0.0);
    tm1[0] = 1.0;                       // T_0
    if (nn > 1) tj[1] = 1.0;            // T_1
    mono[0] += cheb[0];
    if (nn > 1) mono[1] += cheb[1];
    for (int j = 2; j < nn; ++j) {
      std::fill(tn.begin(), tn.end(), 0.0);
      for (int i = 0; i + 1 < nn; ++i) tn[i + 1] += 2.0 * tj[i];
      for (int i = 0; i < nn; ++i) tn[i] -= tm1[i];
      for (int i = 0; i < nn; ++i) mono[i] += cheb[j] * tn[i];
      tm1 = tj;
      tj = tn;
    }
    for (int i = 0; i < nn; ++i) coef[t * nn + i] = float(mono[i]);
  }
  // tap J-1-t at s is tap t at -s (the window is even and the nodes symmetric): make the table say so
  // exactly, as the kernels evaluate the pair from tap t's coefficients
  for (int t = 0; t < J / 2; ++t)
    for (int i = 0; i < nn; ++i) coef[(J - 1 - t) * nn + i] = (i % 2 ? -1.0f : 1.0f) * coef[t * nn + i];
}

// Daubechies extremal-phase scaling filter db_p by spectral factorisation:
// the roots y_j of P(y) = sum_{k<p} C(p-1+k, k) y^k (Durand-Kerner, then Newton polish, in long
// double) give z + 1/z = 2 - 4 y_j; keeping |z| < 1, (1 + z)^p prod (z - z_j) is expanded and
// h[k] is the coefficient of z^(2p-1-k), scaled to sum sqrt(2).
bool daubechies(int p, double* h) {
  typedef long double R;
  typedef std::complex<R> C;
  if (p < 1 || p > 20) return false;
  std::vector<R> P(p);
  for (int k = 0; k < p; ++k) {
    R c = 1;  // C(p-1+k, k)
    for (int i = 1; i <= k; ++i) c = c * R(p - 1 + i) / R(i);
    P[k] = c;
  }
  const int deg = p - 1;
  std::vector<C> roots(deg);
  auto evalP = [&](C y) {
    C acc = P[deg];
    for (int k = deg - 1; k >= 0; --k) acc = acc * y + P[k];
    return acc;
  };
  auto evaldP = [&](C y) {
    C acc = R(deg) * P[deg];
    for (int k = deg - 1; k >= 1; --k) acc = acc * y + R(k) * P[k];
    return acc;
  };
  if (deg > 0) {
    const C seed(R(0.4L), R(0.9L));
    C pw(1, 0);
    for (int i = 0; i < deg; ++i) {
      roots[i] = pw;
      pw *= seed;
    }
    for (int it = 0; it < 2000; ++it) {
      R change = 0;
      for (int i = 0; i < deg; ++i) {
        C den = P[deg];
        for (int j = 0; j < deg; ++j)
          if (j != i) den *= (roots[i] - roots[j]);
        const C step = evalP(roots[i]) / den;
        roots[i] -= step;
        change = std::max(change, std::abs(step));
      }
      if (change < 1e-30L) break;
    }
    for (int i = 0; i < deg; ++i)
      for (int it = 0; it < 5; ++it) {
        const C d = evaldP(roots[i]);
        if (std::abs(d) == 0) break;
        roots[i] -= evalP(roots[i]) / d;
      }
  }
  std::vector<C> poly(1, C(1, 0));  // increasing powers of z
  auto mulfac = [&](C c0, C c1) {   // multiply by (c0 + c1 z)
    std::vector<C> nx(poly.size() + 1, C(0, 0));
    for (size_t i = 0; i < poly.size(); ++i) {
      nx[i] += poly[i] * c0;
      nx[i + 1] += poly[i] * c1;
    }
    poly.swap(nx);
  };
  for (int i = 0; i < p; ++i) mulfac(C(1, 0), C(1, 0));
  for (int i = 0; i < deg; ++i) {
    const C s = R(2) - R(4) * roots[i];
    const C disc = std::sqrt(s * s - R(4));
    C za = (s + disc) / R(2), zb = (s - disc) / R(2);
    const C z = std::abs(za) < 1 ? za : zb;
    mulfac(-z, C(1, 0));
  }
  R tot = 0;
  for (auto& c : poly) tot += c.real();
  const R scale = std::sqrt(R(2)) / tot;
  for (int k = 0; k < 2 * p; ++k) h[k] = double(poly[2 * p - 1 - k].real() * scale);
  return true;
}

void fft_twiddles(int L, std::vector<float2>& tw) {
  tw.resize(L);
  for (int m = 0; m < L; ++m) {
    const double a = 2.0 * M_PI * double(m) / double(L);
    tw[m] = make_float2(float(std::cos(a)), float(-std::sin(a)));  // exp(-2 pi i m / L)
  }
}

}  // namespace sh
