// Device helpers shared by the plan build and the field evaluation: element geometry,
// the quadrature table layout and the Burton-Miller double-layer kernel.
#pragma once

#include "common.hpp"

namespace fmbem {

constexpr double kPi = 3.14159265358979323846;
constexpr double kFourPi = 4.0 * kPi;

// ---------------------------------------------------------------------------
// device: quadrature tables  t in [0,1], w = Gauss weight / 2 (per [0,1] map)
//   layout: q=4 at 0, q=8 at 4, q=16 at 12 (28 entries)
// ---------------------------------------------------------------------------
__device__ inline int quad_off(int q) { return q == 4 ? 0 : (q == 8 ? 4 : 12); }

struct Geo {
  double a[3], b[3], c[3], cen[3], nrm[3], longest, area;
};

__device__ inline Geo load_geo(const double* g, int j) {
  Geo e;
  const double* p = g + (size_t)j * 18;
  for (int i = 0; i < 3; ++i) {
    e.a[i] = p[i];
    e.b[i] = p[3 + i];
    e.c[i] = p[6 + i];
    e.cen[i] = p[9 + i];
    e.nrm[i] = p[12 + i];
  }
  e.longest = p[15];
  e.area = p[16];
  return e;
}

__device__ inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Burton-Miller double-layer kernel dG/dn_y + alpha d2G/dn_x dn_y at x, y (r = x - y)
__device__ inline double2 bm_kernel(const double* r, const double* nx, const double* ny, double k,
                                    double2 alpha, bool hyper) {
  const double R2 = dot3(r, r);
  const double R = sqrt(R2);
  double sn, cs;
  sincos(k * R, &sn, &cs);
  const double2 E = make_double2(cs / kFourPi, sn / kFourPi);
  const double rny = dot3(r, ny);
  const double iR3 = 1.0 / (R2 * R);
  // (1 - ikR)
  const double2 one_m = make_double2(1.0, -k * R);
  double2 dny = cmul<double>(E, one_m);
  dny = cscale<double>(dny, rny * iR3);
  if (!hyper) return dny;
  const double rnx = dot3(r, nx);
  const double nxny = dot3(nx, ny);
  // (3 - 3ikR - k^2R^2)
  const double2 three = make_double2(3.0 - k * k * R2, -3.0 * k * R);
  double2 t1 = cscale<double>(one_m, nxny * iR3);
  double2 t2 = cscale<double>(three, rnx * rny * iR3 / R2);
  double2 d2 = cmul<double>(E, csub<double>(t1, t2));
  return cadd<double>(dny, cmul<double>(alpha, d2));
}

}  // namespace fmbem
