// Host-side float64 tables: Kaiser-Bessel kernel, Daubechies filters, FFT twiddles.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace sh {

double bessel_i0(double x);
double kb_beta(int J, int alpha);
double kb_window(double t, int J, double beta);
double kb_transform(double xi, int J, double beta);
void kb_tap_polys(int J, double beta, int deg, float* coef);
bool daubechies(int p, double* h);
void fft_twiddles(int L, std::vector<float2>& tw);

}  // namespace sh
