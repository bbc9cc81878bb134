// Special functions for the multipole operators, host + device, FP64.
//
// Spherical Bessel functions: j_n by its power series for small arguments,
// Miller's backward recurrence in the transition region and the forward
// recurrence where it is stable (n < z); y_n by the forward recurrence.
// Associated Legendre functions in the semi-normalised form
//   N_n^m(x) = sqrt((n-m)!/(n+m)!) P_n^m(x)   (no Condon-Shortley phase)
// and Q_n^m = N_n^m / sin(theta) (m >= 1), both by the standard three-term
// recurrences in n; Q keeps the angular derivatives finite on the polar axis.
// Harmonics: Y_n^m = (-1)^m N_n^m(cos theta) e^{i m phi} (m >= 0),
// Y_n^{-m} = (-1)^m conj(Y_n^m), so that sum_m Y_n^m(a) conj(Y_n^m(b)) = P_n(a.b).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace fmbem {

// j_0 .. j_nmax at z > 0
__host__ __device__ inline void sph_j_all(int nmax, double z, double* j) {
  if (!(z > 0.0)) {
    j[0] = 1.0;
    for (int n = 1; n <= nmax; ++n) j[n] = 0.0;
    return;
  }
  if (z < 2.0) {
    // power series: j_n(z) = z^n/(2n+1)!! sum_k (-z^2/2)^k / (k! (2n+3)(2n+5)...(2n+2k+1))
    double zn = 1.0, df = 1.0;  // z^n, (2n+1)!!
    const double h = -0.5 * z * z;
    for (int n = 0; n <= nmax; ++n) {
      if (n > 0) { zn *= z; df *= (2.0 * n + 1.0); }
      double term = 1.0, sum = 1.0;
      for (int k = 1; k < 40; ++k) {
        term *= h / (k * (2.0 * n + 2.0 * k + 1.0));
        sum += term;
        if (fabs(term) < 1e-18 * fabs(sum)) break;
      }
      j[n] = zn / df * sum;
    }
    return;
  }
  const double s = sin(z), c = cos(z);
  const double j0 = s / z, j1 = s / (z * z) - c / z;
  if (z > nmax + 1.0) {
    j[0] = j0;
    if (nmax >= 1) j[1] = j1;
    for (int n = 1; n < nmax; ++n) j[n + 1] = (2.0 * n + 1.0) / z * j[n] - j[n - 1];
    return;
  }
  // Miller: f_{L+1} = 0, f_L = tiny, f_{n-1} = (2n+1)/z f_n - f_{n+1}
  const int L = nmax + 30 + (int)z;
  double fp1 = 0.0, f = 1e-250, f0 = 0.0, f1 = 0.0;
  for (int n = L; n >= 1; --n) {
    const double fm1 = (2.0 * n + 1.0) / z * f - fp1;
    fp1 = f;
    f = fm1;  // f = f_{n-1}
    if (n - 1 <= nmax) j[n - 1] = f;
    if (n - 1 == 0) f0 = f;
    if (n - 1 == 1) f1 = f;
  }
  const double scale = (fabs(j0) >= fabs(j1)) ? j0 / f0 : j1 / f1;
  for (int n = 0; n <= nmax; ++n) j[n] *= scale;
}

// y_0 .. y_nmax at z > 0 (forward recurrence)
__host__ __device__ inline void sph_y_all(int nmax, double z, double* y) {
  const double s = sin(z), c = cos(z);
  y[0] = -c / z;
  if (nmax >= 1) y[1] = -c / (z * z) - s / z;
  for (int n = 1; n < nmax; ++n) y[n + 1] = (2.0 * n + 1.0) / z * y[n] - y[n - 1];
}

// N_n^m(x), n = m..nmax, into out[n] (entries n < m untouched); s = sqrt(1-x^2)
__host__ __device__ inline void legendre_N_col(int m, int nmax, double x, double s, double* out) {
  double pmm = 1.0;
  for (int i = 1; i <= m; ++i) pmm *= sqrt((2.0 * i - 1.0) / (2.0 * i)) * s;
  if (m > nmax) return;
  out[m] = pmm;
  if (m + 1 > nmax) return;
  double p1 = x * sqrt(2.0 * m + 1.0) * pmm;
  out[m + 1] = p1;
  double p0 = pmm;
  for (int n = m + 2; n <= nmax; ++n) {
    const double pn = ((2.0 * n - 1.0) * x * p1 - sqrt((double)(n - 1) * (n - 1) - (double)m * m) * p0) /
                      sqrt((double)n * n - (double)m * m);
    out[n] = pn;
    p0 = p1;
    p1 = pn;
  }
}

// Q_n^m(x) = N_n^m / s for m >= 1, n = m..nmax (finite at s = 0)
__host__ __device__ inline void legendre_Q_col(int m, int nmax, double x, double s, double* out) {
  double qmm = sqrt(0.5);
  for (int i = 2; i <= m; ++i) qmm *= sqrt((2.0 * i - 1.0) / (2.0 * i)) * s;
  if (m > nmax) return;
  out[m] = qmm;
  if (m + 1 > nmax) return;
  double q1 = x * sqrt(2.0 * m + 1.0) * qmm;
  out[m + 1] = q1;
  double q0 = qmm;
  for (int n = m + 2; n <= nmax; ++n) {
    const double qn = ((2.0 * n - 1.0) * x * q1 - sqrt((double)(n - 1) * (n - 1) - (double)m * m) * q0) /
                      sqrt((double)n * n - (double)m * m);
    out[n] = qn;
    q0 = q1;
    q1 = qn;
  }
}

}  // namespace fmbem
