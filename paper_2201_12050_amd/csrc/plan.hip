// Plan build: near-field blocks S_d, P2M (V0), L2P (U0), and the per-bin M2L
// symbols Lambda of the circulant embedding of K, all on the device in FP64.
//
// Discretisation (Sec. 2.1, eq. (bm); rigid surface, dp/dn = 0), collocation at
// centroids of flat triangles, normal into the scatterer:
//   A[i,j] = 1/2 delta_ij + int_{Delta_j} [dG/dn_y + alpha d2G/dn_x dn_y](x_i, y) dA(y)
// Quadrature rule (fixed so that independent implementations agree):
//   non-self: Duffy rule collapsed at the first vertex, q x q Gauss-Legendre points,
//             q = 16 / 8 / 4 for |x - centroid_j| < L_j / < 3 L_j / otherwise
//             (L_j = longest edge of element j);
//   self:     dG/dn_y = 0 on a flat element; the hypersingular part is the
//             Hadamard finite part, (1/4pi)[FP int R^-3 dA] in closed form plus
//             (1/4pi) int [e^{ikR}(1-ikR) - 1] R^-3 dA with a 16 x 16 Duffy rule on
//             each sub-triangle (x, v_a, v_b) collapsed at the collocation point x.
//
// Multipole operators (Sec. 3.1, eq. (greenFMM) with argument k|x|; Appendix A):
//   V0[(n,m), b] = int_{Delta_b} d/dn_y conj(I_n^m(y)) dA        (8 x 8 Duffy rule)
//   U0[a, (n,m)] = (ik/4pi)(2n+1)[conj(I_n^m(x_a)) + alpha d/dn_x conj(I_n^m(x_a))]
//   K_d[(n,m),(n',m')] = (2n'+1)(-1)^{m+m'} sum_l (2l+1) i^{n-n'+l}
//                        (n n' l;0 0 0)(n n' l;m m' -m-m') O_l^{m+m'}(d*pitch)
//   with l over max(|m+m'|,|n-n'|) <= l <= n+n', n+n'-l even (eqs. (m2l), (wigner)).
//
// Lambda (Sec. 2.4, eq. (blockDiagonal); Sec. 3.5) is the DFT over the cell grid
// of the first block column of the circulant embedding of K.  Because every
// entry of K_d is a fixed linear combination of the O_l^mu(d*pitch), the build
// transforms the (2n_t+1)^2 scalar fields O_l^mu over the grid instead of the
// p^2 entries of K_d, and forms Lambda_b from the transformed fields per bin.
// The products of the two 3j symbols are computed as Gaunt integrals,
//   (n n' l;0 0 0)(n n' l;m m' -m-m') = 1/2 int_{-1}^{1} Yt_n^m Yt_{n'}^{m'} Yt_l^{-m-m'} dx,
// with Yt the theta-part of Y, by Gauss-Legendre quadrature that is exact for
// the polynomial integrand.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>

#include "common.hpp"
#include "geom.hpp"
#include "specfun.hpp"

namespace fmbem {


// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
void gauss_legendre_host(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= q; ++j) {
        const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (q == 1) { p0 = 1.0; p1 = z; }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int j = 2; j <= q; ++j) {
      const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    if (q == 1) { p0 = 1.0; p1 = z; }
    dp = q * (z * p1 - p0) / (z * z - 1.0);
    x[q - 1 - i] = z;  // ascending
    w[q - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// finite-part self term of the hypersingular kernel on the element's own surface
__device__ double2 hyper_self(const Geo& e, double k, const QuadTab& Q) {
  const double* x = e.cen;
  const double* V[3] = {e.a, e.b, e.c};
  double fp = 0.0;
  for (int s = 0; s < 3; ++s) {
    const double* p = V[s];
    const double* q = V[(s + 1) % 3];
    double ed[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
    const double L = sqrt(dot3(ed, ed));
    for (int i = 0; i < 3; ++i) ed[i] /= L;
    double px[3] = {p[0] - x[0], p[1] - x[1], p[2] - x[2]};
    double qx[3] = {q[0] - x[0], q[1] - x[1], q[2] - x[2]};
    const double tp = dot3(px, ed), tq = dot3(qx, ed);
    double perp[3] = {px[0] - tp * ed[0], px[1] - tp * ed[1], px[2] - tp * ed[2]};
    const double h = sqrt(dot3(perp, perp));
    fp -= (tq / sqrt(dot3(qx, qx)) - tp / sqrt(dot3(px, px))) / h;
  }
  // weakly singular remainder: (1/4pi) int [e^{ikR}(1-ikR) - 1] / R^3 dA
  double re = 0.0, im = 0.0;
  const int o = quad_off(16);
  for (int s = 0; s < 3; ++s) {
    const double* p = V[s];
    const double* q = V[(s + 1) % 3];
    double e1[3] = {p[0] - x[0], p[1] - x[1], p[2] - x[2]};
    double e2[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
    double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double jac = sqrt(dot3(cr, cr));
    for (int ia = 0; ia < 16; ++ia) {
      const double u = Q.t[o + ia];
      const double wu = Q.w[o + ia] * u * jac;
      for (int ib = 0; ib < 16; ++ib) {
        const double v = Q.t[o + ib];
        double d[3];
        for (int i = 0; i < 3; ++i) d[i] = u * (e1[i] + v * e2[i]);
        const double R = sqrt(dot3(d, d));
        const double z = k * R;
        double sn, cs;
        sincos(z, &sn, &cs);
        const double sh = sin(0.5 * z);
        const double gr = -2.0 * sh * sh + z * sn;  // Re[e^{iz}(1-iz)] - 1
        const double gi = sn - z * cs;              // Im[e^{iz}(1-iz)]
        const double wt = wu * Q.w[o + ib] / (R * R * R);
        re += wt * gr;
        im += wt * gi;
      }
    }
  }
  return make_double2((fp + re) / kFourPi, im / kFourPi);
}

// int over the flat triangle with first vertex a, edges ba = b - a and cb = c - b (Duffy rule
// collapsed at a, q x q points, q by the distance from x to the centroid) of the kernel at x
// (ca = c - a for the Jacobian)
__device__ inline double2 elem_integral(const double* x, const double* nx, const double* a, const double* ba,
                                       const double* cb, const double* ca, const double* cen, double longest,
                                       const double* ny, double k, double2 alpha, int hyper, const QuadTab& Q) {
  double dc[3] = {x[0] - cen[0], x[1] - cen[1], x[2] - cen[2]};
  const double dist = sqrt(dot3(dc, dc));
  const int q = dist < longest ? 16 : (dist < 3.0 * longest ? 8 : 4);
  const int o = quad_off(q);
  double cr[3] = {ba[1] * ca[2] - ba[2] * ca[1], ba[2] * ca[0] - ba[0] * ca[2], ba[0] * ca[1] - ba[1] * ca[0]};
  const double jac = sqrt(dot3(cr, cr));
  double re = 0.0, im = 0.0;
  for (int ia = 0; ia < q; ++ia) {
    const double u = Q.t[o + ia];
    const double wu = Q.w[o + ia] * u * jac;
    for (int ib = 0; ib < q; ++ib) {
      const double v = Q.t[o + ib];
      double r[3];
      for (int t = 0; t < 3; ++t) r[t] = x[t] - (a[t] + u * (ba[t] + v * cb[t]));
      const double2 kv = bm_kernel(r, nx, ny, k, alpha, hyper != 0);
      const double wt = wu * Q.w[o + ib];
      re += wt * kv.x;
      im += wt * kv.y;
    }
  }
  return make_double2(re, im);
}

// S_d[i][j] for collocation element ex (index i) and source element ey (index j) of the cell
// shifted by sh = -d * pitch
__device__ inline double2 near_entry(const Geo& ex, const Geo& ey, bool same, int o0, int o1, int o2,
                                     const double* sh, double k, double2 alpha, int hyper, const QuadTab& Q) {
  if (o0 == 0 && o1 == 0 && o2 == 0 && same) {
    double2 val = make_double2(0.5, 0.0);
    if (hyper) val = cadd<double>(val, cmul<double>(alpha, hyper_self(ex, k, Q)));
    return val;
  }
  double a[3], ba[3], cb[3], ca[3], cen[3];
  for (int t = 0; t < 3; ++t) {
    a[t] = ey.a[t] + sh[t];
    ba[t] = ey.b[t] - ey.a[t];
    cb[t] = ey.c[t] - ey.b[t];
    ca[t] = ey.c[t] - ey.a[t];
    cen[t] = ey.cen[t] + sh[t];
  }
  return elem_integral(ex.cen, ex.nrm, a, ba, cb, ca, cen, ey.longest, ey.nrm, k, alpha, hyper, Q);
}

// entries of the P2P blocks of the multilevel near field, one per thread in block order (the
// block of entry idx found by bisection over the block offsets)
__global__ void ml_p2p_kernel(const double* __restrict__ geom, const P2pBlock* __restrict__ blk, int nblk,
                              long long base, long long total, const int* __restrict__ perm, double p0, double p1,
                              double p2, double k, double2 alpha, int hyper, QuadTab Q, double2* __restrict__ out) {
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    int lo = 0, hi = nblk - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (blk[mid].off - base <= idx) lo = mid;
      else hi = mid - 1;
    }
    const P2pBlock b = blk[lo];
    const long long r = idx - (b.off - base);
    const int i = (int)(r / b.ns), j = (int)(r - (long long)i * b.ns);
    const int o0 = b.sd % 3 - 1, o1 = (b.sd / 3) % 3 - 1, o2 = b.sd / 9 - 1;
    const double sh[3] = {-o0 * p0, -o1 * p1, -o2 * p2};
    const int ei = perm[b.te0 + i], ej = perm[b.se0 + j];
    out[b.off + r - base] = near_entry(load_geo(geom, ei), load_geo(geom, ej), ei == ej, o0, o1, o2, sh, k, alpha,
                                       hyper, Q);
  }
}

// one entry S_d[i][j] per thread; entries ordered (d, i, j) with j fastest.  Half-space:
// img = 1 (plane parallel to the periodic axes) adds R_p times the image block to every near
// block: the source element of the shifted cell mirrored in z = zg, vertices (a, c, b) so that
// its normal is the mirrored normal; img = 2 (the image sub-plan of a lattice periodic along z)
// holds the image block alone, for offset (d0, d1, e) the source cell shifted by (e + zbase) p2
// along z before the mirroring (zbase = M3 - 1: e indexes the input reversed along z).
__global__ void assemble_near_kernel(const double* __restrict__ geom, int n, const int* __restrict__ offs, int n_near,
                            double p0, double p1, double p2, double k, double2 alpha, int hyper, QuadTab Q,
                            int img, int zbase, double zg, double2 rp, double2* __restrict__ S64,
                            float2* __restrict__ S32) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nn = (size_t)n * n;
  if (idx >= nn * n_near) return;
  const int d = (int)(idx / nn);
  const size_t rem = idx - (size_t)d * nn;
  const int i = (int)(rem / n);
  const int j = (int)(rem - (size_t)i * n);
  const int o0 = offs[3 * d], o1 = offs[3 * d + 1], o2 = offs[3 * d + 2];
  const double sh[3] = {-o0 * p0, -o1 * p1, -o2 * p2};
  const Geo ex = load_geo(geom, i);
  const Geo ey = load_geo(geom, j);
  double2 val = make_double2(0.0, 0.0);
  if (img != 2) val = near_entry(ex, ey, i == j, o0, o1, o2, sh, k, alpha, hyper, Q);
  if (img) {
    // mirrored element (a, c, b): z -> 2 zg - z after the lattice shift
    const double shz = img == 2 ? (o2 + zbase) * p2 : sh[2];
    double a[3] = {ey.a[0] + sh[0], ey.a[1] + sh[1], 2.0 * zg - (ey.a[2] + shz)};
    double c[3] = {ey.c[0] + sh[0], ey.c[1] + sh[1], 2.0 * zg - (ey.c[2] + shz)};
    double b[3] = {ey.b[0] + sh[0], ey.b[1] + sh[1], 2.0 * zg - (ey.b[2] + shz)};
    // the mirrored triangle (a, c, b): edges c - a and b - c, Jacobian from b - a
    double ca[3], bc[3], ba[3];
    for (int t = 0; t < 3; ++t) {
      ca[t] = c[t] - a[t];
      bc[t] = b[t] - c[t];
      ba[t] = b[t] - a[t];
    }
    const double cen[3] = {ey.cen[0] + sh[0], ey.cen[1] + sh[1], 2.0 * zg - (ey.cen[2] + shz)};
    const double ny[3] = {ey.nrm[0], ey.nrm[1], -ey.nrm[2]};
    const double2 w = elem_integral(ex.cen, ex.nrm, a, ca, bc, ba, cen, ey.longest, ny, k, alpha, hyper, Q);
    val = cadd<double>(val, cmul<double>(rp, w));
  }
  S64[idx] = val;
  if (S32) S32[idx] = make_float2((float)val.x, (float)val.y);
}

// gradient of conj(I_n^m) at v (cell-local), dotted with nrm, for fixed m >= 0, n = m..nt;
// also returns conj(I_n^m) values.  Spherical-coordinate form with Q = N / sin(theta).
struct RegularWork {
  double jn[24], jd[24], N[24], Q[24], N1[24];
};

__device__ inline void regular_m(const double* v, const double* nrm, double k, int nt, int m, RegularWork& W,
                                 double2* cI, double2* dn) {
  const double rho2 = v[0] * v[0] + v[1] * v[1];
  const double r = sqrt(rho2 + v[2] * v[2]);
  const double rho = sqrt(rho2);
  const double ct = r > 0 ? v[2] / r : 1.0;
  const double st = r > 0 ? rho / r : 0.0;
  const double cp = rho > 0 ? v[0] / rho : 1.0;
  const double sp = rho > 0 ? v[1] / rho : 0.0;
  const double z = k * r;
  sph_j_all(nt + 1, z, W.jn);
  // j_n' = j_{n-1} - (n+1)/z j_n ; j_0' = -j_1
  W.jd[0] = -W.jn[1];
  for (int n = 1; n <= nt; ++n) W.jd[n] = W.jn[n - 1] - (n + 1.0) / z * W.jn[n];
  legendre_N_col(m, nt, ct, st, W.N);
  if (m >= 1) legendre_Q_col(m, nt, ct, st, W.Q);
  else legendre_Q_col(1, nt, ct, st, W.N1);  // N_n^1 = st * Q_n^1 for the m = 0 theta-derivative
  // e^{i m phi}
  double er = 1.0, ei = 0.0;
  for (int t = 0; t < m; ++t) {
    const double nr = er * cp - ei * sp;
    ei = er * sp + ei * cp;
    er = nr;
  }
  const double sg = (m & 1) ? -1.0 : 1.0;
  const double rh[3] = {st * cp, st * sp, ct};
  const double th[3] = {ct * cp, ct * sp, -st};
  const double ph[3] = {-sp, cp, 0.0};
  const double nr_ = dot3(nrm, rh), nt_ = dot3(nrm, th), np_ = dot3(nrm, ph);
  for (int n = m; n <= nt; ++n) {
    // theta part of Y and its derivative, and Y / sin(theta)
    const double yv = sg * W.N[n];
    double dth;
    double ys;  // Y/sin(theta) (real factor)
    if (m >= 1) {
      const double qm1 = (n - 1 >= m) ? W.Q[n - 1] : 0.0;
      dth = sg * (n * ct * W.Q[n] - sqrt((double)(n + m) * (n - m)) * qm1);
      ys = sg * W.Q[n];
    } else {
      dth = (n >= 1) ? -sqrt((double)n * (n + 1)) * st * W.N1[n] : 0.0;
      ys = 0.0;
    }
    // conj(I) = j_n * yv * e^{-i m phi}
    cI[n] = make_double2(W.jn[n] * yv * er, -W.jn[n] * yv * ei);
    // grad conj(I): conj of [k j' Y rhat + j/r dY/dth that + j/r i m Y/s phat]
    const double jr = r > 0 ? W.jn[n] / r : 0.0;
    const double gr_re = k * W.jd[n] * yv * nr_ + jr * dth * nt_;
    // real factors times e^{-i m phi} for the first two terms; third term: conj(i m ys e^{i m phi})
    //   = -i m ys e^{-i m phi}
    const double t3 = jr * m * ys * np_;
    // (gr_re) * (er - i ei) + (-i t3) * (er - i ei) = gr_re er - t3 ei + i(-gr_re ei - t3 er)
    dn[n] = make_double2(gr_re * er - t3 * ei, -gr_re * ei - t3 * er);
  }
}

// V0: one wave per (element b, m >= 0), one lane per point of the 8x8 Duffy rule; the
// lane contributions are summed by a fixed shuffle tree.
__device__ inline double wave_sum64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// cen (optional): expansion centre of every element ([n][3], default the origin); pos (optional):
// column of every element (default its index)
__global__ __launch_bounds__(64) void p2m_kernel(const double* __restrict__ geom, int n, int nt, double k,
                                                 QuadTab Qt, const double* __restrict__ isig,
                                                 double2* __restrict__ V0, const double* __restrict__ cen,
                                                 const int* __restrict__ pos) {
  const int b = blockIdx.x / (nt + 1);
  const int m = blockIdx.x - b * (nt + 1);
  const int lane = threadIdx.x;
  const Geo e = load_geo(geom, b);
  double ba[3], cb[3], ca[3];
  for (int t = 0; t < 3; ++t) { ba[t] = e.b[t] - e.a[t]; cb[t] = e.c[t] - e.b[t]; ca[t] = e.c[t] - e.a[t]; }
  double cr[3] = {ba[1] * ca[2] - ba[2] * ca[1], ba[2] * ca[0] - ba[0] * ca[2], ba[0] * ca[1] - ba[1] * ca[0]};
  const double jac = sqrt(dot3(cr, cr));
  const int o = quad_off(8);
  const int ia = lane / 8, ib = lane % 8;
  const double u = Qt.t[o + ia], v = Qt.t[o + ib];
  const double wt = Qt.w[o + ia] * u * jac * Qt.w[o + ib];
  double y[3];
  for (int t = 0; t < 3; ++t) y[t] = e.a[t] + u * (ba[t] + v * cb[t]) - (cen ? cen[3 * b + t] : 0.0);
  const int col = pos ? pos[b] : b;
  RegularWork W;
  double2 cI[21], dn[21];
  regular_m(y, e.nrm, k, nt, m, W, cI, dn);
  const double sg = (m & 1) ? -1.0 : 1.0;
  for (int nn = m; nn <= nt; ++nn) {
    const double re = wave_sum64(wt * dn[nn].x), im = wave_sum64(wt * dn[nn].y);
    if (lane == 0) {
      V0[(size_t)(nn * nn + nn + m) * n + col] = cscale<double>(make_double2(re, im), isig[nn]);
      // conj(I_n^{-m}) = (-1)^m I_n^m => its gradient is (-1)^m conj(grad conj(I_n^m))
      if (m > 0) V0[(size_t)(nn * nn + nn - m) * n + col] = cscale<double>(make_double2(sg * re, -sg * im), isig[nn]);
    }
  }
}

// U0: one thread per (element a, m >= 0), at the centroid (cen, pos: as for p2m_kernel, pos the row)
__global__ void l2p_kernel(const double* __restrict__ geom, int n, int nt, double k, double2 alpha,
                           const double* __restrict__ isig, double2* __restrict__ U0, const double* __restrict__ cen,
                           const int* __restrict__ pos) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= n * (nt + 1)) return;
  const int a = tid / (nt + 1);
  const int m = tid - a * (nt + 1);
  const Geo e = load_geo(geom, a);
  double x[3];
  for (int t = 0; t < 3; ++t) x[t] = e.cen[t] - (cen ? cen[3 * a + t] : 0.0);
  const size_t row = pos ? pos[a] : a;
  RegularWork W;
  double2 cI[21], dn[21];
  regular_m(x, e.nrm, k, nt, m, W, cI, dn);
  const int p = (nt + 1) * (nt + 1);
  const double sg = (m & 1) ? -1.0 : 1.0;
  for (int nn = m; nn <= nt; ++nn) {
    const double f = k / kFourPi * (2.0 * nn + 1.0) * isig[nn];
    const double2 ik = make_double2(0.0, f);  // (ik/4pi)(2n+1)/sigma_n
    double2 vp = cadd<double>(cI[nn], cmul<double>(alpha, dn[nn]));
    U0[row * p + nn * nn + nn + m] = cmul<double>(ik, vp);
    if (m > 0) {
      // conj(I_n^{-m}) = (-1)^m conj(conj(I_n^m)); gradient likewise
      double2 vm = cadd<double>(cconj<double>(cI[nn]), cmul<double>(alpha, cconj<double>(dn[nn])));
      vm = cscale<double>(vm, sg);
      U0[row * p + nn * nn + nn - m] = cmul<double>(ik, vm);
    }
  }
}

// O_l^mu(d * pitch) on the circulant grid, zero at near offsets and padding gaps.
// one thread per (bin, mu >= 0); output [bin][(2nt+1)^2]
// the z component of offset d is (d2 + zbase) p2 - zsub (zbase = zsub = 0 for the direct part; the
// image offsets of the half-space shift it, computed in the same order as the host's near list);
// mask_near: 1 zeroes the near offsets (Chebyshev radius r per axis), 0 keeps them all (image
// blocks that are all far), 2 zeroes those with |d0| <= r0, |d1| <= r1 and |z offset| <
// (r2 + 1) p2 (the image blocks of a lattice periodic along z)
__global__ void ogrid_kernel(int B, int N0, int N1, int N2, int M0, int M1, int M2, int r0, int r1, int r2,
                             double p0, double p1, double p2, double k, int L, int zbase, double zsub,
                             int mask_near, double2* __restrict__ O) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= B * (L + 1)) return;
  const int bin = tid / (L + 1);
  const int mu = tid - bin * (L + 1);
  const int P2 = (L + 1) * (L + 1);
  const int b0 = bin % N0, b1 = (bin / N0) % N1, b2 = bin / (N0 * N1);
  auto off = [](int b, int N, int M, bool& gap) {
    gap = false;
    if (b <= M - 1) return b;
    if (b >= N - (M - 1)) return b - N;
    gap = true;
    return 0;
  };
  bool g0, g1, g2;
  const int d0 = off(b0, N0, M0, g0), d1 = off(b1, N1, M1, g1), d2 = off(b2, N2, M2, g2);
  // product and difference rounded separately, as on the host (no fused multiply-add), so that
  // the near / far decision at |z| = (r2 + 1) p2 agrees with the near list
  const double D[3] = {d0 * p0, d1 * p1, __dsub_rn(__dmul_rn((double)(d2 + zbase), p2), zsub)};
  const bool near = mask_near == 2 ? (abs(d0) <= r0 && abs(d1) <= r1 && fabs(D[2]) < (r2 + 1) * p2)
                                   : mask_near && (abs(d0) <= r0 && abs(d1) <= r1 && abs(d2) <= r2);
  double2* out = O + (size_t)bin * P2;
  if (g0 || g1 || g2 || near) {
    for (int l = mu; l <= L; ++l) {
      out[l * l + l + mu] = make_double2(0, 0);
      if (mu > 0) out[l * l + l - mu] = make_double2(0, 0);
    }
    return;
  }
  const double rho2 = D[0] * D[0] + D[1] * D[1];
  const double r = sqrt(rho2 + D[2] * D[2]);
  const double rho = sqrt(rho2);
  const double ct = D[2] / r, st = rho / r;
  const double cp = rho > 0 ? D[0] / rho : 1.0, sp = rho > 0 ? D[1] / rho : 0.0;
  double jl[42], yl[42], Nl[42];
  sph_j_all(L, k * r, jl);
  sph_y_all(L, k * r, yl);
  legendre_N_col(mu, L, ct, st, Nl);
  double er = 1.0, ei = 0.0;
  for (int t = 0; t < mu; ++t) {
    const double nr = er * cp - ei * sp;
    ei = er * sp + ei * cp;
    er = nr;
  }
  const double sg = (mu & 1) ? -1.0 : 1.0;
  for (int l = mu; l <= L; ++l) {
    const double2 h = make_double2(jl[l], yl[l]);
    // Y_l^mu = (-1)^mu N e^{i mu phi};  Y_l^{-mu} = N e^{-i mu phi}
    out[l * l + l + mu] = cmul<double>(h, make_double2(sg * Nl[l] * er, sg * Nl[l] * ei));
    if (mu > 0) out[l * l + l - mu] = cmul<double>(h, make_double2(Nl[l] * er, -Nl[l] * ei));
  }
}

// Lambda'_c[j][i] (column-major per canonical bin c) = s^{n+n'}/B * sum_terms coef * Ohat_bin(c)[oidx].
// Half-space (Ohi != nullptr): plus R_p (-1)^{n'+m'} sum_terms coef * Ohi_bin(c)[oidx], the image
// translations acting on the reflected moments D_z V0 x (Appendix A, eq. (greenFMMhalfspace)).
__global__ void lambda_kernel(const double2* __restrict__ Oh, const double2* __restrict__ Ohi, double2 rp, int P2,
                              int p, const int* __restrict__ pairs, const int* __restrict__ ptr,
                              const double2* __restrict__ coef, const int* __restrict__ oidx,
                              const double* __restrict__ sig, const int* __restrict__ nof, double invB, int ldp,
                              double2* __restrict__ L64, float2* __restrict__ L32) {
  extern __shared__ double2 so[];
  double2* soi = so + P2;
  const int slot = blockIdx.y;
  const int bin = pairs[2 * slot];
  for (int t = threadIdx.x; t < P2; t += blockDim.x) {
    so[t] = Oh ? Oh[(size_t)bin * P2 + t] : make_double2(0.0, 0.0);
    if (Ohi) soi[t] = Ohi[(size_t)bin * P2 + t];
  }
  __syncthreads();
  const size_t pp = (size_t)p * p;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < pp; e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / p);   // column (n', m')
    const int i = (int)(e - (size_t)j * p);  // row (n, m)
    const int te = i * p + j;
    double re = 0.0, im = 0.0;
    for (int t = ptr[te]; t < ptr[te + 1]; ++t) {
      const double2 c = coef[t];
      const double2 o = so[oidx[t]];
      re += c.x * o.x - c.y * o.y;
      im += c.x * o.y + c.y * o.x;
    }
    if (Ohi) {
      double ri = 0.0, ii = 0.0;
      for (int t = ptr[te]; t < ptr[te + 1]; ++t) {
        const double2 c = coef[t];
        const double2 o = soi[oidx[t]];
        ri += c.x * o.x - c.y * o.y;
        ii += c.x * o.y + c.y * o.x;
      }
      const int nj = nof[j], mj = j - nj * nj - nj;
      const double sg = ((nj + mj) & 1) ? -1.0 : 1.0;
      re += sg * (rp.x * ri - rp.y * ii);
      im += sg * (rp.x * ii + rp.y * ri);
    }
    const double f = sig[nof[i]] * sig[nof[j]] * invB;
    const double2 v = make_double2(re * f, im * f);
    const size_t o = ((size_t)slot * p + j) * ldp + i;
    L64[o] = v;
    if (L32) L32[o] = make_float2((float)v.x, (float)v.y);
    if (i == p - 1 && ldp > p) {  // zero the padding row of the column
      L64[o + 1] = make_double2(0, 0);
      if (L32) L32[o + 1] = make_float2(0.f, 0.f);
    }
  }
}

__global__ void cast_kernel(const double2* __restrict__ a, float2* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

hipError_t cast_launch(const double2* a, float2* b, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(cast_kernel, dim3(4096), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

// incident fields: b = p_inc + alpha dp_inc/dn at every collocation point
// p_inc and dp_inc/dn of a plane wave (complex amplitude a, unit direction s) or a monopole at s
__device__ inline void incident_at(const double* x, const double* nx, const double* s, int point, double k,
                                   double2 a, double2& pv, double2& dp) {
  if (!point) {
    double sn, cs;
    sincos(k * dot3(s, x), &sn, &cs);
    pv = cmul<double>(a, make_double2(cs, sn));
    dp = cmul<double>(make_double2(0.0, k * dot3(s, nx)), pv);
  } else {
    const double d[3] = {x[0] - s[0], x[1] - s[1], x[2] - s[2]};
    const double R = sqrt(dot3(d, d));
    double sn, cs;
    sincos(k * R, &sn, &cs);
    pv = cmul<double>(a, make_double2(cs / R, sn / R));
    // dp/dn = A e^{ikR} (ikR - 1)/R^2 * (d.n)/R
    const double f = dot3(d, nx) / (R * R * R);
    dp = cmul<double>(cmul<double>(a, make_double2(cs * f, sn * f)), make_double2(-1.0, k * R));
  }
}

// half != 0: plus R_p times the image of the incident field in the plane z = zg, i.e. a plane
// wave of direction (s0, s1, -s2) and amplitude R_p A e^{2ik zg s2}, or a monopole R_p A at the
// mirrored source (Sec. 2.1, eq. (green3dHalf))
__global__ void incident_kernel(const double* __restrict__ geom, int n, int C, int g0, int g1, double p0,
                                double p1, double p2, double k, double2 alpha, int R, const double* __restrict__ src,
                                int point, double amp, int half, double zg, double2 rp, double2* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t N = (size_t)n * C;
  if (idx >= N * R) return;
  const int r = (int)(idx / N);
  const size_t rem = idx - (size_t)r * N;
  const int c = (int)(rem / n);
  const int i = (int)(rem - (size_t)c * n);
  const double* g = geom + (size_t)i * 18;
  const int i1 = c % g0, i2 = (c / g0) % g1, i3 = c / (g0 * g1);
  const double x[3] = {g[9] + i1 * p0, g[10] + i2 * p1, g[11] + i3 * p2};
  const double nx[3] = {g[12], g[13], g[14]};
  const double* s = src + 3 * r;
  double2 pv, dp;
  incident_at(x, nx, s, point, k, make_double2(amp, 0.0), pv, dp);
  if (half) {
    double2 a = cscale<double>(rp, amp), pi, di;
    double si[3] = {s[0], s[1], point ? 2.0 * zg - s[2] : -s[2]};
    if (!point) {
      double sn, cs;
      sincos(2.0 * k * zg * s[2], &sn, &cs);
      a = cmul<double>(a, make_double2(cs, sn));
    }
    incident_at(x, nx, si, point, k, a, pi, di);
    pv = cadd<double>(pv, pi);
    dp = cadd<double>(dp, di);
  }
  out[idx] = cadd<double>(pv, cmul<double>(alpha, dp));
}

// Exact periodic BEM (Sec. 2.2 eq. (toeplitzBEM), Sec. 2.4 eq. (blockDiagonal)): the first block
// column of the circulant embedding holds the exact block S_d at bin (d mod N) for every offset of
// the lattice; S [nd][n n] -> G [bin][n n] (G zeroed first)
__global__ void place_blocks_kernel(const double2* __restrict__ S, const int* __restrict__ bins, int nd, size_t nn,
                                    double2* __restrict__ G) {
  const size_t total = (size_t)nd * nn;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t d = e / nn, r = e - d * nn;
    G[(size_t)bins[d] * nn + r] = S[e];
  }
}

// Lambda_b = G_b / B transposed to the column-major per-bin layout (column stride ldp) of the
// M2L products, FP64 and (optionally) FP32
__global__ void exact_lambda_kernel(const double2* __restrict__ G, int B, int n, int ldp, double inv,
                                    double2* __restrict__ L64, float2* __restrict__ L32) {
  const size_t nn = (size_t)n * n, total = (size_t)B * nn;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t b = e / nn, r = e - b * nn;
    const int i = (int)(r / n), j = (int)(r - (size_t)i * n);
    const double2 v = G[e];
    const double2 o = make_double2(v.x * inv, v.y * inv);
    const size_t dst = (b * n + j) * ldp + i;
    L64[dst] = o;
    if (L32) L32[dst] = make_float2((float)o.x, (float)o.y);
  }
}

// n x n identity (the P2M and L2P maps of the exact operator), FP64 and (optionally) FP32
__global__ void identity_kernel(double2* __restrict__ I64, float2* __restrict__ I32, int n) {
  const size_t total = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const double v = (e / n == e % n) ? 1.0 : 0.0;
    I64[e] = make_double2(v, 0.0);
    if (I32) I32[e] = make_float2((float)v, 0.0f);
  }
}

// ---------------------------------------------------------------------------
// host: plan creation
// ---------------------------------------------------------------------------
#define FM_CHECK(expr)                         \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return e_;           \
  } while (0)

hipError_t plan_alloc(Plan& P, void** ptr, size_t bytes) {
  FM_CHECK(hipMalloc(ptr, bytes));
  P.allocations.push_back(*ptr);
  P.resident += bytes;
  return hipSuccess;
}

static void free_list(std::vector<void*>& v) {
  for (void* p : v) hipFree(p);
  v.clear();
}

// theta part of the harmonics at Gauss nodes: table [l][mu + l][node], l <= L
void theta_table(int L, const std::vector<double>& x, std::vector<double>& tab) {
  const int q = (int)x.size();
  const int W = 2 * L + 1;
  tab.assign((size_t)(L + 1) * W * q, 0.0);
  std::vector<double> col(L + 1);
  for (int i = 0; i < q; ++i) {
    const double s = std::sqrt(std::max(0.0, 1.0 - x[i] * x[i]));
    for (int mu = 0; mu <= L; ++mu) {
      legendre_N_col(mu, L, x[i], s, col.data());
      const double sg = (mu & 1) ? -1.0 : 1.0;
      for (int l = mu; l <= L; ++l) {
        tab[((size_t)l * W + (L + mu)) * q + i] = sg * col[l];  // Yt_l^mu
        tab[((size_t)l * W + (L - mu)) * q + i] = col[l];       // Yt_l^{-mu} = (-1)^mu Yt_l^mu
      }
    }
  }
}

struct M2LTable {
  std::vector<int> ptr, oidx;
  std::vector<double2> coef;
};

static void m2l_table(int nt, M2LTable& T) {
  const int p = (nt + 1) * (nt + 1);
  const int L = 2 * nt;
  std::vector<double> gx, gw;
  gauss_legendre_host(2 * nt + 2, gx, gw);
  std::vector<double> tab;
  theta_table(L, gx, tab);
  const int q = (int)gx.size();
  const int W = 2 * L + 1;
  auto yt = [&](int l, int mu) { return &tab[((size_t)l * W + (L + mu)) * q]; };
  T.ptr.assign((size_t)p * p + 1, 0);
  T.coef.clear();
  T.oidx.clear();
  static const double ire[4] = {1, 0, -1, 0}, iim[4] = {0, 1, 0, -1};
  for (int n = 0; n <= nt; ++n)
    for (int m = -n; m <= n; ++m)
      for (int n2 = 0; n2 <= nt; ++n2)
        for (int m2 = -n2; m2 <= n2; ++m2) {
          const int e = (n * n + n + m) * p + (n2 * n2 + n2 + m2);
          const int mu = m + m2;
          int lo = std::max(std::abs(mu), std::abs(n - n2));
          if ((n + n2 - lo) & 1) ++lo;
          for (int l = lo; l <= n + n2; l += 2) {
            const double* a = yt(n, m);
            const double* b = yt(n2, m2);
            const double* c = yt(l, -mu);
            double g = 0.0;
            for (int i = 0; i < q; ++i) g += gw[i] * a[i] * b[i] * c[i];
            g *= 0.5;
            const double f = (2.0 * n2 + 1.0) * (((m + m2) & 1) ? -1.0 : 1.0) * (2.0 * l + 1.0) * g;
            const int ip = (((n - n2 + l) % 4) + 4) % 4;
            T.coef.push_back(make_double2(f * ire[ip], f * iim[ip]));
            T.oidx.push_back(l * l + l + mu);
          }
          T.ptr[e + 1] = (int)T.coef.size();
        }
}

void plan_release(Plan* P) {
  if (!P) return;
  if (P->img) {
    plan_release(P->img);
    P->img = nullptr;
  }
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(P->device);
  for (auto& m : P->prof.marks) {
    hipEventSynchronize(m.second.second);
    hipEventDestroy(m.second.first);
    hipEventDestroy(m.second.second);
  }
  for (hipEvent_t e : P->prof.pool) hipEventDestroy(e);
  if (P->aux) {
    hipStreamSynchronize(P->aux);
    hipStreamDestroy(P->aux);
  }
  if (P->ev_fork) hipEventDestroy(P->ev_fork);
  if (P->ev_join) hipEventDestroy(P->ev_join);
  free_list(P->allocations);
  hipSetDevice(cur);
  delete P;
}

hipError_t ml_assemble_launch(const Plan& P, int nt, const std::vector<double>& cen, const std::vector<double>& isig,
                              const std::vector<P2pBlock>& blocks, long long entries, double2* ops, long long oV,
                              long long oU, hipStream_t s) {
  const int n = P.n;
  std::vector<void*> scratch;
  auto salloc = [&](void** ptr, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(ptr, bytes);
    if (e == hipSuccess) scratch.push_back(*ptr);
    return e;
  };
  double *d_cen = nullptr, *d_isig = nullptr;
  P2pBlock* d_blk = nullptr;
  hipError_t err = hipSuccess;
  do {
    if ((err = salloc((void**)&d_cen, cen.size() * sizeof(double)))) break;
    if ((err = salloc((void**)&d_isig, isig.size() * sizeof(double)))) break;
    if ((err = salloc((void**)&d_blk, std::max<size_t>(1, blocks.size()) * sizeof(P2pBlock)))) break;
    hipMemcpyAsync(d_cen, cen.data(), cen.size() * sizeof(double), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d_isig, isig.data(), isig.size() * sizeof(double), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d_blk, blocks.data(), blocks.size() * sizeof(P2pBlock), hipMemcpyHostToDevice, s);
    const double2 alpha = make_double2(P.alpha_re, P.alpha_im);
    const int hyper = (P.alpha_re != 0.0 || P.alpha_im != 0.0) ? 1 : 0;
    const int th = n * (nt + 1);
    hipLaunchKernelGGL(p2m_kernel, dim3(th), dim3(64), 0, s, P.geom, n, nt, P.k, P.quad, d_isig, ops + oV, d_cen,
                       P.ml->pos);
    hipLaunchKernelGGL(l2p_kernel, dim3((th + 63) / 64), dim3(64), 0, s, P.geom, n, nt, P.k, alpha, d_isig, ops + oU,
                       d_cen, P.ml->pos);
    if (entries > 0) {
      const long long base = blocks[0].off;
      const unsigned g = (unsigned)std::min<long long>((entries + 255) / 256, 1 << 16);
      hipLaunchKernelGGL(ml_p2p_kernel, dim3(g), dim3(256), 0, s, P.geom, d_blk, (int)blocks.size(), base, entries,
                         P.ml->perm, P.pitch[0], P.pitch[1], P.pitch[2], P.k, alpha, hyper, P.quad, ops + base);
    }
    if ((err = hipGetLastError())) break;
    err = hipStreamSynchronize(s);  // the host tables must outlive their copies
  } while (0);
  const hipError_t e2 = hipStreamSynchronize(s);
  free_list(scratch);
  return err ? err : e2;
}

// Exact periodic BEM plan: every block S_d (|d_a| <= M_a - 1) integrated like the near blocks,
// placed at bin (d mod N) of the zeroed grid, the grid transformed (forward DFT over every bin,
// n^2 channels), Lambda_b = that transform / B per bin; V0 = U0 = I (p = n); no near blocks.
static hipError_t exact_build(Plan& P, const QuadTab& Q, double2 alpha, int hyper, bool want32, hipStream_t s) {
  const int n = P.n;
  const size_t nn = (size_t)n * n;
  // offsets of the lattice and their bins
  std::vector<int> offs, bins;
  for (int d2 = -(P.grid[2] - 1); d2 <= P.grid[2] - 1; ++d2)
    for (int d1 = -(P.grid[1] - 1); d1 <= P.grid[1] - 1; ++d1)
      for (int d0 = -(P.grid[0] - 1); d0 <= P.grid[0] - 1; ++d0) {
        offs.push_back(d0);
        offs.push_back(d1);
        offs.push_back(d2);
        const int b0 = (d0 + P.fft[0]) % P.fft[0], b1 = (d1 + P.fft[1]) % P.fft[1], b2 = (d2 + P.fft[2]) % P.fft[2];
        bins.push_back(b0 + P.fft[0] * (b1 + P.fft[1] * b2));
      }
  const int nd = (int)bins.size();
  FM_CHECK(plan_alloc(P, &P.S[0], sizeof(double2)));  // no near blocks
  if (want32) FM_CHECK(plan_alloc(P, &P.S[1], sizeof(float2)));
  std::vector<void*> scratch;
  auto salloc = [&](void** ptr, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(ptr, bytes);
    if (e == hipSuccess) scratch.push_back(*ptr);
    return e;
  };
  hipError_t err = hipSuccess;
  do {
    int *d_offs = nullptr, *d_bins = nullptr;
    double2 *Sall = nullptr, *G = nullptr;
    if ((err = salloc((void**)&d_offs, offs.size() * sizeof(int))) != hipSuccess) break;
    if ((err = salloc((void**)&d_bins, bins.size() * sizeof(int))) != hipSuccess) break;
    if ((err = salloc((void**)&Sall, (size_t)nd * nn * sizeof(double2))) != hipSuccess) break;
    if ((err = salloc((void**)&G, (size_t)P.B * nn * sizeof(double2))) != hipSuccess) break;
    hipMemcpyAsync(d_offs, offs.data(), offs.size() * sizeof(int), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d_bins, bins.data(), bins.size() * sizeof(int), hipMemcpyHostToDevice, s);
    hipMemsetAsync(G, 0, (size_t)P.B * nn * sizeof(double2), s);
    const size_t total = (size_t)nd * nn;
    hipLaunchKernelGGL(assemble_near_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, P.geom, n, d_offs,
                       nd, P.pitch[0], P.pitch[1], P.pitch[2], P.k, alpha, hyper, Q, 0, 0, 0.0, make_double2(0, 0),
                       Sall, (float2*)nullptr);
    hipLaunchKernelGGL(place_blocks_kernel, dim3(4096), dim3(256), 0, s, Sall, d_bins, nd, nn, G);
    if ((err = hipGetLastError()) != hipSuccess) break;
    if ((err = grid_dft_launch<double>(G, (int)nn, P.fft, P.fft, false, false, s)) != hipSuccess) break;
    // every bin is its own canonical bin (the exact blocks have no D-symmetry pairing)
    std::vector<int> canon(P.B), pairs(2 * (size_t)P.B);
    for (int b = 0; b < P.B; ++b) {
      canon[b] = b;
      pairs[2 * b] = b;
      pairs[2 * b + 1] = -1;
    }
    P.Bc = P.B;
    if ((err = plan_alloc(P, (void**)&P.d_canon, P.B * sizeof(int))) != hipSuccess) break;
    if ((err = plan_alloc(P, (void**)&P.d_pairs, pairs.size() * sizeof(int))) != hipSuccess) break;
    hipMemcpyAsync(P.d_canon, canon.data(), P.B * sizeof(int), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(P.d_pairs, pairs.data(), pairs.size() * sizeof(int), hipMemcpyHostToDevice, s);
    const int ldp = lambda_ld(n);
    const size_t nl = (size_t)P.B * n * ldp;
    if ((err = plan_alloc(P, &P.Lam[0], nl * sizeof(double2))) != hipSuccess) break;
    if (want32 && (err = plan_alloc(P, &P.Lam[1], nl * sizeof(float2))) != hipSuccess) break;
    if (ldp != n) {
      hipMemsetAsync(P.Lam[0], 0, nl * sizeof(double2), s);
      if (want32) hipMemsetAsync(P.Lam[1], 0, nl * sizeof(float2), s);
    }
    hipLaunchKernelGGL(exact_lambda_kernel, dim3(4096), dim3(256), 0, s, G, P.B, n, ldp, 1.0 / P.B,
                       (double2*)P.Lam[0], (float2*)P.Lam[1]);
    // V0 = U0 = I (n x n)
    if ((err = plan_alloc(P, &P.V0[0], nn * sizeof(double2))) != hipSuccess) break;
    if ((err = plan_alloc(P, &P.U0[0], nn * sizeof(double2))) != hipSuccess) break;
    if (want32 && (err = plan_alloc(P, &P.V0[1], nn * sizeof(float2))) != hipSuccess) break;
    if (want32 && (err = plan_alloc(P, &P.U0[1], nn * sizeof(float2))) != hipSuccess) break;
    hipLaunchKernelGGL(identity_kernel, dim3(256), dim3(256), 0, s, (double2*)P.V0[0], (float2*)P.V0[1], n);
    hipLaunchKernelGGL(identity_kernel, dim3(256), dim3(256), 0, s, (double2*)P.U0[0], (float2*)P.U0[1], n);
    err = hipGetLastError();
  } while (0);
  // host tables must outlive the async copies; the scratch buffers are freed after the stream drains
  hipError_t e2 = hipStreamSynchronize(s);
  free_list(scratch);
  if (err == hipSuccess) err = e2;
  return err;
}

static hipError_t plan_build(Plan& P, const std::vector<double>& geo, hipStream_t s) {
  const int n = P.n;
  // geometry (an image sub-plan shares its parent's)
  if (P.parent) {
    P.geom = P.parent->geom;
  } else {
    FM_CHECK(plan_alloc(P, (void**)&P.geom, geo.size() * sizeof(double)));
    FM_CHECK(hipMemcpyAsync(P.geom, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice, s));
  }
  FM_CHECK(plan_alloc(P, (void**)&P.d_near, std::max<size_t>(1, P.near_off.size()) * sizeof(int)));
  FM_CHECK(hipMemcpyAsync(P.d_near, P.near_off.data(), P.near_off.size() * sizeof(int), hipMemcpyHostToDevice, s));
  // quadrature table
  QuadTab& Q = P.quad;
  {
    int o = 0;
    for (int q : {4, 8, 16}) {
      std::vector<double> x, w;
      gauss_legendre_host(q, x, w);
      for (int i = 0; i < q; ++i) {
        Q.t[o + i] = 0.5 * (x[i] + 1.0);
        Q.w[o + i] = 0.5 * w[i];
      }
      o += q;
    }
  }
  const bool want32 = (P.precisions & (1u << FMBEM_FP32)) != 0;
  // DFT matrices of the axes for the GEMM schedule of the grid DFT (Sec. 2.4, the DFT over the
  // grid as products with the Fourier matrices): forward [N][M] (pruned input), inverse [M][N]
  // (cropped output, conjugate kernel; the 1/B of the inverse is folded into Lambda)
  std::vector<double2> fm64[6];
  std::vector<float2> fm32[6];
  auto dft_mats = [&]() -> hipError_t {
    for (int a = 0; a < 3; ++a) {
      const int Nn = P.fft[a], Mm = P.grid[a];
      if (Nn <= 1 || Nn > kDftGemmMaxOut) continue;
      for (int dir = 0; dir < 2; ++dir) {
        const int rows = dir == 0 ? Nn : Mm, cols = dir == 0 ? Mm : Nn;
        const double sgn = dir == 0 ? -1.0 : 1.0;
        const int slot = 3 * dir + a;
        std::vector<double2>& h = fm64[slot];
        h.resize((size_t)rows * cols);
        for (int k = 0; k < rows; ++k)
          for (int j = 0; j < cols; ++j) {
            const double ang = 2.0 * M_PI * (double)(((long long)k * j) % Nn) / Nn;
            h[(size_t)k * cols + j] = make_double2(std::cos(ang), sgn * std::sin(ang));
          }
        FM_CHECK(plan_alloc(P, &P.dftF[0][slot], h.size() * sizeof(double2)));
        FM_CHECK(hipMemcpyAsync(P.dftF[0][slot], h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice, s));
        if (want32) {
          std::vector<float2>& h32 = fm32[slot];
          h32.resize(h.size());
          for (size_t i = 0; i < h.size(); ++i) h32[i] = make_float2((float)h[i].x, (float)h[i].y);
          FM_CHECK(plan_alloc(P, &P.dftF[1][slot], h32.size() * sizeof(float2)));
          FM_CHECK(hipMemcpyAsync(P.dftF[1][slot], h32.data(), h32.size() * sizeof(float2), hipMemcpyHostToDevice,
                                  s));
        }
      }
    }
    return hipSuccess;
  };
  if (P.parent) {
    for (int a = 0; a < 6; ++a) {
      P.dftF[0][a] = P.parent->dftF[0][a];
      P.dftF[1][a] = P.parent->dftF[1][a];
    }
  } else {
    // the host tables must outlive their copies, also when a step fails
    const hipError_t e1 = dft_mats();
    const hipError_t e2 = hipStreamSynchronize(s);
    FM_CHECK(e1);
    FM_CHECK(e2);
  }
  const double2 alpha = make_double2(P.alpha_re, P.alpha_im);
  const int hyper = (P.alpha_re != 0.0 || P.alpha_im != 0.0) ? 1 : 0;
  if (P.exact) return exact_build(P, Q, alpha, hyper, want32, s);
  // near blocks
  const size_t ns = (size_t)P.n_near * n * n;
  FM_CHECK(plan_alloc(P, &P.S[0], std::max<size_t>(1, ns) * sizeof(double2)));
  if (want32) FM_CHECK(plan_alloc(P, &P.S[1], std::max<size_t>(1, ns) * sizeof(float2)));
  if (ns > 0) {
    const size_t blocks = (ns + 255) / 256;
    hipLaunchKernelGGL(assemble_near_kernel, dim3((unsigned)blocks), dim3(256), 0, s, P.geom, n, P.d_near, P.n_near,
                       P.pitch[0], P.pitch[1], P.pitch[2], P.k, alpha, hyper, Q,
                       P.parent ? 2 : (P.fold && P.img_near ? 1 : 0), P.grid[2] - 1, P.zg,
                       make_double2(P.rp_re, P.rp_im), (double2*)P.S[0], (float2*)P.S[1]);
    FM_CHECK(hipGetLastError());
  }
  // scaling s^n
  const int nt = P.order, p = P.p;
  std::vector<double> sig(nt + 1), isig(nt + 1);
  for (int i = 0; i <= nt; ++i) {
    sig[i] = std::pow(P.scale, i);
    isig[i] = 1.0 / sig[i];
  }
  double* d_sig = nullptr;
  double* d_isig = nullptr;
  std::vector<void*> scratch;
  auto salloc = [&](void** ptr, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(ptr, bytes);
    if (e == hipSuccess) scratch.push_back(*ptr);
    return e;
  };
  hipError_t err = hipSuccess;
  do {
    if ((err = salloc((void**)&d_sig, sig.size() * sizeof(double))) != hipSuccess) break;
    if ((err = salloc((void**)&d_isig, isig.size() * sizeof(double))) != hipSuccess) break;
    hipMemcpyAsync(d_sig, sig.data(), sig.size() * sizeof(double), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d_isig, isig.data(), isig.size() * sizeof(double), hipMemcpyHostToDevice, s);
    // V0, U0 (an image sub-plan shares its parent's)
    if (P.parent) {
      for (int q = 0; q < 2; ++q) {
        P.V0[q] = P.parent->V0[q];
        P.U0[q] = P.parent->U0[q];
      }
    }
    if (!P.parent && (err = plan_alloc(P, &P.V0[0], (size_t)p * n * sizeof(double2))) != hipSuccess) break;
    if (!P.parent && (err = plan_alloc(P, &P.U0[0], (size_t)p * n * sizeof(double2))) != hipSuccess) break;
    if (!P.parent) {
      const int th = n * (nt + 1);
      hipLaunchKernelGGL(p2m_kernel, dim3(th), dim3(64), 0, s, P.geom, n, nt, P.k, Q, d_isig, (double2*)P.V0[0],
                         (const double*)nullptr, (const int*)nullptr);
      hipLaunchKernelGGL(l2p_kernel, dim3((th + 63) / 64), dim3(64), 0, s, P.geom, n, nt, P.k, alpha, d_isig,
                         (double2*)P.U0[0], (const double*)nullptr, (const int*)nullptr);
      if ((err = hipGetLastError()) != hipSuccess) break;
    }
    if (want32 && !P.parent) {
      if ((err = plan_alloc(P, &P.V0[1], (size_t)p * n * sizeof(float2))) != hipSuccess) break;
      if ((err = plan_alloc(P, &P.U0[1], (size_t)p * n * sizeof(float2))) != hipSuccess) break;
      hipLaunchKernelGGL(cast_kernel, dim3(256), dim3(256), 0, s, (const double2*)P.V0[0], (float2*)P.V0[1],
                         (size_t)p * n);
      hipLaunchKernelGGL(cast_kernel, dim3(256), dim3(256), 0, s, (const double2*)P.U0[0], (float2*)P.U0[1],
                         (size_t)p * n);
    }
    if (P.ml && (err = ml_build(P, geo, s)) != hipSuccess) break;
    if (P.n_far == 0) break;
    // O grid -> FFT -> Lambda
    const int L = 2 * nt, P2 = (L + 1) * (L + 1);
    // direct translations (none in an image sub-plan); image translations: target centre minus
    // mirrored source centre, (d0 p0, d1 p1, -2 zg) with the plane parallel to the periodic axes,
    // (d0 p0, d1 p1, (e + M3 - 1) p2 - 2 zg) for offset e of the z-reversed input in a sub-plan
    const bool direct = !P.parent, image = P.fold || P.parent;
    double2 *Og = nullptr, *Ogi = nullptr;
    if (direct && (err = salloc((void**)&Og, (size_t)P.B * P2 * sizeof(double2))) != hipSuccess) break;
    if (image && (err = salloc((void**)&Ogi, (size_t)P.B * P2 * sizeof(double2))) != hipSuccess) break;
    {
      const int th = P.B * (L + 1);
      int rr[3];
      for (int a = 0; a < 3; ++a) rr[a] = P.grid[a] > 1 ? std::min(P.near_radius[a], P.grid[a] - 1) : 0;
      if (direct)
        hipLaunchKernelGGL(ogrid_kernel, dim3((th + 127) / 128), dim3(128), 0, s, P.B, P.fft[0], P.fft[1],
                           P.fft[2], P.grid[0], P.grid[1], P.grid[2], rr[0], rr[1], rr[2], P.pitch[0], P.pitch[1],
                           P.pitch[2], P.k, L, 0, 0.0, 1, Og);
      if (P.fold)
        hipLaunchKernelGGL(ogrid_kernel, dim3((th + 127) / 128), dim3(128), 0, s, P.B, P.fft[0], P.fft[1],
                           P.fft[2], P.grid[0], P.grid[1], P.grid[2], rr[0], rr[1], rr[2], P.pitch[0], P.pitch[1],
                           P.pitch[2], P.k, L, 0, 2.0 * P.zg, P.img_near ? 1 : 0, Ogi);
      if (P.parent)
        hipLaunchKernelGGL(ogrid_kernel, dim3((th + 127) / 128), dim3(128), 0, s, P.B, P.fft[0], P.fft[1],
                           P.fft[2], P.grid[0], P.grid[1], P.grid[2], rr[0], rr[1], P.near_radius[2], P.pitch[0],
                           P.pitch[1], P.pitch[2], P.k, L, P.grid[2] - 1, 2.0 * P.zg, 2, Ogi);
      if ((err = hipGetLastError()) != hipSuccess) break;
    }
    if (direct && (err = grid_dft_launch<double>(Og, P2, P.fft, P.fft, false, false, s)) != hipSuccess) break;
    if (image && (err = grid_dft_launch<double>(Ogi, P2, P.fft, P.fft, false, false, s)) != hipSuccess) break;
    M2LTable T;
    m2l_table(nt, T);
    int *d_ptr = nullptr, *d_oidx = nullptr, *d_nof = nullptr;
    double2* d_coef = nullptr;
    if ((err = salloc((void**)&d_ptr, T.ptr.size() * sizeof(int))) != hipSuccess) break;
    if ((err = salloc((void**)&d_oidx, std::max<size_t>(1, T.oidx.size()) * sizeof(int))) != hipSuccess) break;
    if ((err = salloc((void**)&d_coef, std::max<size_t>(1, T.coef.size()) * sizeof(double2))) != hipSuccess) break;
    std::vector<int> nof(p);
    for (int nn = 0; nn <= nt; ++nn)
      for (int m = -nn; m <= nn; ++m) nof[nn * nn + nn + m] = nn;
    if ((err = salloc((void**)&d_nof, p * sizeof(int))) != hipSuccess) break;
    hipMemcpyAsync(d_ptr, T.ptr.data(), T.ptr.size() * sizeof(int), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d_oidx, T.oidx.data(), T.oidx.size() * sizeof(int), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d_coef, T.coef.data(), T.coef.size() * sizeof(double2), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(d_nof, nof.data(), p * sizeof(int), hipMemcpyHostToDevice, s);
    // canonical bins: linear index not above that of the partner bin -w (without the pairing,
    // every bin is its own canonical bin)
    std::vector<int> canon(P.B), pairs;
    for (int b2 = 0; b2 < P.fft[2]; ++b2)
      for (int b1 = 0; b1 < P.fft[1]; ++b1)
        for (int b0 = 0; b0 < P.fft[0]; ++b0) {
          const int L = b0 + P.fft[0] * (b1 + P.fft[1] * b2);
          const int Lp = !P.paired ? L
                                   : (P.fft[0] - b0) % P.fft[0] +
                                         P.fft[0] * ((P.fft[1] - b1) % P.fft[1] +
                                                     P.fft[1] * ((P.fft[2] - b2) % P.fft[2]));
          if (L > Lp) continue;
          canon[L] = canon[Lp] = (int)(pairs.size() / 2);
          pairs.push_back(L);
          pairs.push_back(Lp == L ? -1 : Lp);
        }
    P.Bc = (int)(pairs.size() / 2);
    if ((err = plan_alloc(P, (void**)&P.d_canon, P.B * sizeof(int))) != hipSuccess) break;
    if ((err = plan_alloc(P, (void**)&P.d_pairs, pairs.size() * sizeof(int))) != hipSuccess) break;
    hipMemcpyAsync(P.d_canon, canon.data(), P.B * sizeof(int), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(P.d_pairs, pairs.data(), pairs.size() * sizeof(int), hipMemcpyHostToDevice, s);
    const int ldp = lambda_ld(p);
    const size_t nl = (size_t)P.Bc * p * ldp;
    if ((err = plan_alloc(P, &P.Lam[0], nl * sizeof(double2))) != hipSuccess) break;
    if (want32 && (err = plan_alloc(P, &P.Lam[1], nl * sizeof(float2))) != hipSuccess) break;
    {
      const int bx = (int)std::min<size_t>(((size_t)p * p + 255) / 256, 64);
      hipLaunchKernelGGL(lambda_kernel, dim3(bx, P.Bc), dim3(256), 2 * P2 * sizeof(double2), s, Og,
                         Ogi, make_double2(P.rp_re, P.rp_im), P2, p, P.d_pairs, d_ptr, d_coef, d_oidx, d_sig, d_nof,
                         1.0 / P.B, ldp, (double2*)P.Lam[0], (float2*)P.Lam[1]);
      if ((err = hipGetLastError()) != hipSuccess) break;
    }
    // host vectors (T) must outlive the async copies
    err = hipStreamSynchronize(s);
  } while (0);
  hipError_t e2 = hipStreamSynchronize(s);
  free_list(scratch);
  if (err == hipSuccess) err = e2;
  return err;
}

}  // namespace fmbem

using namespace fmbem;

// The image part of a half-space lattice periodic along z (block Hankel along z, Sec. 2.3):
// applied to the input reversed along z it is block Toeplitz in (d0, d1, e), e = target - reversed
// source index, so it is a plan of its own over the same grid: near blocks for the image offsets
// within the near range (|d0| <= r0, |d1| <= r1, |(e + M3 - 1) p2 - 2 zg| < (r2 + 1) p2), the
// other image offsets through the multipole chain with the reflected moments (Sec. 3.4,
// Appendix A, eq. (greenFMMhalfspace)); geometry, V0, U0 and the DFT matrices are the parent's.
static hipError_t image_plan_create(Plan& P, const std::vector<double>& geo, hipStream_t s) {
  Plan* I = new (std::nothrow) Plan();
  if (!I) return hipErrorOutOfMemory;
  I->device = P.device;
  I->n = P.n;
  I->C = P.C;
  for (int a = 0; a < 3; ++a) {
    I->grid[a] = P.grid[a];
    I->pitch[a] = P.pitch[a];
    I->near_radius[a] = P.near_radius[a];
    I->fft[a] = P.fft[a];
  }
  I->B = P.B;
  I->k = P.k;
  I->order = P.order;
  I->p = P.p;
  I->p2 = P.p2;
  I->formulation = P.formulation;
  I->alpha_re = P.alpha_re;
  I->alpha_im = P.alpha_im;
  I->precisions = P.precisions;
  I->scale = P.scale;
  I->dft_forced = P.dft_forced;
  for (int a = 0; a < 3; ++a) I->tile_forced[a] = P.tile_forced[a];
  I->parent = &P;
  I->paired = false;
  I->zg = P.zg;
  I->rp_re = P.rp_re;
  I->rp_im = P.rp_im;
  const int M3 = P.grid[2];
  int rr[2];
  for (int a = 0; a < 2; ++a) rr[a] = P.grid[a] > 1 ? std::min(P.near_radius[a], P.grid[a] - 1) : 0;
  int total = 0;
  for (int e3 = -(M3 - 1); e3 <= M3 - 1; ++e3) {
    const double dz = (e3 + M3 - 1) * P.pitch[2] - 2.0 * P.zg;
    const bool znear = std::fabs(dz) < (P.near_radius[2] + 1) * P.pitch[2];
    for (int d1 = -(P.grid[1] - 1); d1 <= P.grid[1] - 1; ++d1)
      for (int d0 = -(P.grid[0] - 1); d0 <= P.grid[0] - 1; ++d0) {
        ++total;
        if (znear && std::abs(d0) <= rr[0] && std::abs(d1) <= rr[1]) {
          I->near_off.push_back(d0);
          I->near_off.push_back(d1);
          I->near_off.push_back(e3);
        }
      }
  }
  I->n_near = (int)I->near_off.size() / 3;
  I->n_far = total - I->n_near;
  hipError_t e = I->n_near > kMaxSeg ? hipErrorInvalidValue : hipSuccess;
  if (e == hipSuccess) e = plan_build(*I, geo, s);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&I->aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&I->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&I->ev_join, hipEventDisableTiming);
  if (e != hipSuccess) {
    plan_release(I);
    return e;
  }
  P.img = I;
  return hipSuccess;
}

extern "C" fmbem_status fmbem_plan_create(const fmbem_cell_mesh* mesh, const fmbem_plan_desc* desc, void* hip_stream,
                                          fmbem_plan* out) {
  if (!mesh || !desc || !out) return FMBEM_ERR_INVALID_ARG;
  *out = nullptr;
  if (mesh->n_vertices < 3 || mesh->n_triangles < 1 || !mesh->vertices || !mesh->triangles)
    return FMBEM_ERR_INVALID_ARG;
  for (int a = 0; a < 3; ++a) {
    if (desc->grid[a] < 1 || !(desc->pitch[a] > 0.0)) return FMBEM_ERR_INVALID_ARG;
    if (desc->near_radius[a] < 0 || desc->near_radius[a] > 3) return FMBEM_ERR_INVALID_ARG;
    if (desc->fft_shape[a] < 0) return FMBEM_ERR_INVALID_ARG;
    if (desc->fft_shape[a] > 0 && desc->fft_shape[a] < 2 * desc->grid[a] - 1) return FMBEM_ERR_INVALID_ARG;
    if (desc->grid[a] > kMaxGridDim || desc->fft_shape[a] > 2 * kMaxGridDim) return FMBEM_ERR_UNSUPPORTED;
  }
  if (!(desc->k > 0.0) || !std::isfinite(desc->k)) return FMBEM_ERR_INVALID_ARG;
  if (desc->exact != 0 && desc->exact != 1) return FMBEM_ERR_INVALID_ARG;
  if (desc->exact == 1 && desc->halfspace != 0) return FMBEM_ERR_UNSUPPORTED;
  if (desc->exact == 0 && (desc->order < 0 || desc->order > 20)) return FMBEM_ERR_INVALID_ARG;
  if (desc->near_levels < 0 || desc->near_levels > 8 || desc->near_order < 0 || desc->near_order > 7)
    return FMBEM_ERR_INVALID_ARG;
  if (desc->near_levels > 0) {
    if (desc->exact != 0 || desc->halfspace != 0) return FMBEM_ERR_UNSUPPORTED;
    for (int a = 0; a < 3; ++a)
      if (desc->near_radius[a] > 1) return FMBEM_ERR_UNSUPPORTED;
  }
  if (desc->formulation != FMBEM_BURTON_MILLER && desc->formulation != FMBEM_CBIE) return FMBEM_ERR_INVALID_ARG;
  if (desc->precisions & ~3u) return FMBEM_ERR_INVALID_ARG;
  if (desc->dft_schedule < FMBEM_DFT_AUTO || desc->dft_schedule > FMBEM_DFT_FFT) return FMBEM_ERR_INVALID_ARG;
  if (desc->halfspace != 0 && desc->halfspace != 1) return FMBEM_ERR_INVALID_ARG;
  for (int a = 0; a < 3; ++a)
    if (desc->tile_shape[a] < 0 || desc->tile_shape[a] > FMBEM_TILE_SHAPES) return FMBEM_ERR_INVALID_ARG;
  if (desc->halfspace == 1) {
    if (!std::isfinite(desc->plane_z) || !std::isfinite(desc->reflection_re) || !std::isfinite(desc->reflection_im))
      return FMBEM_ERR_INVALID_ARG;
    // the surface of every layer stays on one side of the plane (vertices on it allowed)
    double zmin = HUGE_VAL, zmax = -HUGE_VAL;
    for (int v = 0; v < mesh->n_vertices; ++v) {
      zmin = std::min(zmin, mesh->vertices[3 * v + 2]);
      zmax = std::max(zmax, mesh->vertices[3 * v + 2]);
    }
    zmax += (desc->grid[2] - 1) * desc->pitch[2];
    if (!(zmin >= desc->plane_z || zmax <= desc->plane_z)) return FMBEM_ERR_INVALID_ARG;
  }
  const int n = mesh->n_triangles;
  // geometry on the host: a, b, c, centroid, unit normal, longest edge, area
  std::vector<double> geo((size_t)n * 18, 0.0);
  for (int t = 0; t < n; ++t) {
    const int* tri = mesh->triangles + 3 * t;
    double v[3][3];
    for (int c = 0; c < 3; ++c) {
      if (tri[c] < 0 || tri[c] >= mesh->n_vertices) return FMBEM_ERR_INVALID_ARG;
      for (int i = 0; i < 3; ++i) {
        v[c][i] = mesh->vertices[3 * tri[c] + i];
        if (!std::isfinite(v[c][i])) return FMBEM_ERR_INVALID_ARG;
      }
    }
    double e1[3], e2[3], e3[3];
    for (int i = 0; i < 3; ++i) {
      e1[i] = v[1][i] - v[0][i];
      e2[i] = v[2][i] - v[0][i];
      e3[i] = v[2][i] - v[1][i];
    }
    double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double two_a = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    auto len = [](const double* e) { return std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]); };
    const double longest = std::max(std::max(len(e1), len(e3)), len(e2));
    if (!(two_a > 1e-14 * longest * longest)) return FMBEM_ERR_INVALID_ARG;
    double* g = geo.data() + (size_t)t * 18;
    for (int i = 0; i < 3; ++i) {
      g[i] = v[0][i];
      g[3 + i] = v[1][i];
      g[6 + i] = v[2][i];
      g[9 + i] = (v[0][i] + v[1][i] + v[2][i]) / 3.0;
      g[12 + i] = cr[i] / two_a;
    }
    g[15] = longest;
    g[16] = 0.5 * two_a;
  }
  if (desc->near_levels > 0 && !ml_cell_fits(geo, n, desc->pitch, desc->near_levels)) return FMBEM_ERR_UNSUPPORTED;
  Plan* P = new (std::nothrow) Plan();
  if (!P) return FMBEM_ERR_OUT_OF_MEMORY;
  if (hipGetDevice(&P->device) != hipSuccess) {
    delete P;
    return FMBEM_ERR_DEVICE;
  }
  P->n = n;
  P->C = 1;
  for (int a = 0; a < 3; ++a) {
    P->grid[a] = desc->grid[a];
    P->pitch[a] = desc->pitch[a];
    P->near_radius[a] = desc->near_radius[a] == 0 ? 1 : desc->near_radius[a];
    P->C *= desc->grid[a];
    const int need = 2 * desc->grid[a] - 1;
    // any length N >= 2 M - 1 embeds the block Toeplitz product exactly; on lattices with M3 = 1
    // the grid transform runs as FFTs over even lengths (radix 2, 4 or 8 by divisibility), so the
    // default is 2 M there (one bin more per axis than the smallest embedding); 3-D lattices keep
    // 2 M - 1 (the direct pruned axis passes take any length)
    P->fft[a] = desc->fft_shape[a] > 0 ? desc->fft_shape[a] : (desc->grid[2] == 1 ? need + 1 : need);
    if (desc->grid[a] == 1) P->fft[a] = 1;
  }
  P->B = P->fft[0] * P->fft[1] * P->fft[2];
  P->k = desc->k;
  P->exact = desc->exact == 1;
  P->order = P->exact ? 0 : desc->order;
  // exact PBEM: the per-bin blocks act on the element values themselves (p = n)
  P->p = P->exact ? n : (desc->order + 1) * (desc->order + 1);
  P->p2 = (2 * P->order + 1) * (2 * P->order + 1);
  P->formulation = desc->formulation;
  if (desc->formulation == FMBEM_CBIE) {
    P->alpha_re = 0.0;
    P->alpha_im = 0.0;
  } else if (std::isnan(desc->alpha_re) && std::isnan(desc->alpha_im)) {
    P->alpha_re = 0.0;
    P->alpha_im = -1.0 / desc->k;
  } else {
    P->alpha_re = desc->alpha_re;
    P->alpha_im = desc->alpha_im;
  }
  P->precisions = desc->precisions == 0 ? 1u : desc->precisions;
  P->dft_forced = desc->dft_schedule - 1;
  for (int a = 0; a < 3; ++a) P->tile_forced[a] = desc->tile_shape[a] - 1;
  // near offsets (Chebyshev radius, axes with a single cell dropped)
  int rr[3];
  for (int a = 0; a < 3; ++a) rr[a] = P->grid[a] > 1 ? std::min(P->near_radius[a], P->grid[a] - 1) : 0;
  for (int d2 = -rr[2]; d2 <= rr[2]; ++d2)
    for (int d1 = -rr[1]; d1 <= rr[1]; ++d1)
      for (int d0 = -rr[0]; d0 <= rr[0]; ++d0) {
        P->near_off.push_back(d0);
        P->near_off.push_back(d1);
        P->near_off.push_back(d2);
      }
  if (P->exact) {
    P->near_off.clear();  // every block goes through the transformed column
    P->paired = false;
  }
  P->n_near = (int)P->near_off.size() / 3;
  if (P->n_near > kMaxSeg) {
    delete P;
    return FMBEM_ERR_UNSUPPORTED;
  }
  P->n_far = (2 * P->grid[0] - 1) * (2 * P->grid[1] - 1) * (2 * P->grid[2] - 1) - P->n_near;
  if (desc->near_levels > 0) {
    // the near offsets stay out of the far field but have no dense blocks
    P->ml = std::make_shared<MlData>();
    P->ml->levels = desc->near_levels;
    P->ml->order = desc->near_order > 0 ? desc->near_order : std::max(1, std::min(desc->order, 7));
    P->ml->p = (P->ml->order + 1) * (P->ml->order + 1);
    P->near_off.clear();
    P->n_near = 0;
  }
  if (desc->halfspace == 1) {
    P->half = true;
    P->zg = desc->plane_z;
    P->rp_re = desc->reflection_re;
    P->rp_im = desc->reflection_im;
    if (P->grid[2] == 1) {
      // plane parallel to every periodic axis: image blocks near for the near offsets when the
      // mirrored cells lie within the near range along z (|2 zg| < (r + 1) pitch_z), all through
      // the multipole chain otherwise, folded into this plan
      P->fold = true;
      P->paired = false;
      P->img_near = std::fabs(2.0 * P->zg) < (P->near_radius[2] + 1) * P->pitch[2];
      P->n_far_img = (2 * P->grid[0] - 1) * (2 * P->grid[1] - 1) - (P->img_near ? P->n_near : 0);
      P->n_far += P->n_far_img;
    }
  }
  // scaling: s = k * (largest distance of a vertex from the cell centre), at most 1
  double rmax = 0.0;
  for (int v = 0; v < mesh->n_vertices; ++v) {
    const double* x = mesh->vertices + 3 * v;
    rmax = std::max(rmax, std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]));
  }
  P->scale = P->exact ? 1.0 : std::min(1.0, std::max(1e-3, P->k * rmax));
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e = plan_build(*P, geo, s);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming);
  if (e == hipSuccess && P->half && !P->fold) e = image_plan_create(*P, geo, s);
  if (e != hipSuccess) {
    plan_release(P);
    return to_status(e);
  }
  *out = reinterpret_cast<fmbem_plan>(P);
  return FMBEM_OK;
}

extern "C" fmbem_status fmbem_plan_destroy(fmbem_plan plan) {
  if (!plan) return FMBEM_ERR_INVALID_ARG;
  plan_release(reinterpret_cast<Plan*>(plan));
  return FMBEM_OK;
}

extern "C" fmbem_status fmbem_plan_query(fmbem_plan plan, fmbem_plan_info* out) {
  if (!plan || !out) return FMBEM_ERR_INVALID_ARG;
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  out->n_dof_cell = P.n;
  out->n_cells = P.C;
  out->n_dof = (int64_t)P.n * P.C;
  out->p = P.p;
  for (int a = 0; a < 3; ++a) out->fft_shape[a] = P.fft[a];
  out->n_near = P.n_near;
  out->n_far = P.n_far + (P.img ? P.img->n_far : 0);
  out->precisions = P.precisions;
  out->resident_bytes = P.resident + (P.img ? P.img->resident : 0);
  out->workspace_bytes_per_rhs[0] = matvec_workspace_bytes_per_rhs(P, FMBEM_FP64);
  out->workspace_bytes_per_rhs[1] = matvec_workspace_bytes_per_rhs(P, FMBEM_FP32);
  out->scale = P.scale;
  out->near_levels = P.ml ? P.ml->levels : 0;
  out->near_order = P.ml ? P.ml->order : 0;
  out->near_boxes = P.ml ? P.ml->boxes : 0;
  out->near_m2l_pairs = P.ml ? P.ml->m2l_pairs : 0;
  out->near_p2p_entries = P.ml ? P.ml->p2p_entries : 0;
  out->near_macs_per_rhs = P.ml ? P.ml->macs_per_rhs : 0.0;
  out->near_max_tasks = P.ml ? P.ml->max_tasks : 0;
  return FMBEM_OK;
}

extern "C" fmbem_status fmbem_plan_export(fmbem_plan plan, int32_t what, void* host, size_t host_bytes) {
  if (!plan || !host) return FMBEM_ERR_INVALID_ARG;
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  const int n = P.n, p = P.p;
  int cur = 0;
  hipGetDevice(&cur);
  if (hipSetDevice(P.device) != hipSuccess) return FMBEM_ERR_DEVICE;
  fmbem_status st = FMBEM_OK;
  std::vector<double2> tmp;
  switch (what) {
    case 0: {
      const size_t bytes = (size_t)P.n_near * n * n * sizeof(double2);
      if (host_bytes < bytes) { st = FMBEM_ERR_INVALID_ARG; break; }
      st = to_status(hipMemcpy(host, P.S[0], bytes, hipMemcpyDeviceToHost));
      break;
    }
    case 1:
    case 2: {
      const size_t cnt = (size_t)p * n;
      if (host_bytes < cnt * sizeof(double2)) { st = FMBEM_ERR_INVALID_ARG; break; }
      double2* h = reinterpret_cast<double2*>(host);
      st = to_status(hipMemcpy(h, what == 1 ? P.V0[0] : P.U0[0], cnt * sizeof(double2), hipMemcpyDeviceToHost));
      if (st != FMBEM_OK) break;
      for (size_t e = 0; e < cnt; ++e) {
        const int idx = what == 1 ? (int)(e / n) : (int)(e % p);
        const int nn = (int)std::floor(std::sqrt((double)idx) + 1e-9);
        const double sg = std::pow(P.scale, nn);
        h[e].x *= sg;
        h[e].y *= sg;
      }
      break;
    }
    case 3: {
      const size_t pp = (size_t)p * p;
      const size_t cnt = (size_t)P.B * pp;
      if (host_bytes < cnt * sizeof(double2)) { st = FMBEM_ERR_INVALID_ARG; break; }
      if (!P.Lam[0]) {
        std::memset(host, 0, cnt * sizeof(double2));
        break;
      }
      const size_t ldp = (size_t)lambda_ld(p);
      tmp.resize((size_t)P.Bc * p * ldp);
      st = to_status(hipMemcpy(tmp.data(), P.Lam[0], tmp.size() * sizeof(double2), hipMemcpyDeviceToHost));
      if (st != FMBEM_OK) break;
      std::vector<int> canon(P.B), pairs(2 * (size_t)P.Bc);
      st = to_status(hipMemcpy(canon.data(), P.d_canon, P.B * sizeof(int), hipMemcpyDeviceToHost));
      if (st == FMBEM_OK)
        st = to_status(hipMemcpy(pairs.data(), P.d_pairs, pairs.size() * sizeof(int), hipMemcpyDeviceToHost));
      if (st != FMBEM_OK) break;
      double2* h = reinterpret_cast<double2*>(host);
      std::vector<int> nof(p);
      for (int nn = 0; nn <= P.order; ++nn)
        for (int m = -nn; m <= nn; ++m) nof[nn * nn + nn + m] = nn;
      for (int b = 0; b < P.B; ++b) {
        // a non-canonical bin holds D Lambda D of its canonical partner
        const int c = canon[b];
        const bool flip = pairs[2 * c] != b;
        for (int j = 0; j < p; ++j)
          for (int i = 0; i < p; ++i) {
            double f = P.B / (std::pow(P.scale, nof[i]) * std::pow(P.scale, nof[j]));
            if (flip && ((nof[i] + nof[j]) & 1)) f = -f;
            const double2 v = tmp[((size_t)c * p + j) * ldp + i];
            h[(size_t)b * pp + (size_t)i * p + j] = make_double2(v.x * f, v.y * f);
          }
      }
      break;
    }
    case 4: {
      const size_t bytes = P.near_off.size() * sizeof(int);
      if (host_bytes < bytes) { st = FMBEM_ERR_INVALID_ARG; break; }
      std::memcpy(host, P.near_off.data(), bytes);
      break;
    }
    default:
      st = FMBEM_ERR_INVALID_ARG;
  }
  hipSetDevice(cur);
  return st;
}

static fmbem_status incident(fmbem_plan plan, int32_t R, const double* src, double amp, void* b, void* hs,
                             int point) {
  if (!plan || !src || !b || R < 1 || !std::isfinite(amp)) return FMBEM_ERR_INVALID_ARG;
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  for (int i = 0; i < 3 * R; ++i)
    if (!std::isfinite(src[i])) return FMBEM_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(hs);
  double* d_src = nullptr;
  if (hipMallocAsync((void**)&d_src, 3 * R * sizeof(double), s) != hipSuccess) return FMBEM_ERR_OUT_OF_MEMORY;
  hipError_t e = hipMemcpyAsync(d_src, src, 3 * R * sizeof(double), hipMemcpyHostToDevice, s);
  const size_t total = (size_t)P.n * P.C * R;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(incident_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, P.geom, P.n, P.C,
                       P.grid[0], P.grid[1], P.pitch[0], P.pitch[1], P.pitch[2], P.k,
                       make_double2(P.alpha_re, P.alpha_im), R, d_src, point, amp, P.half ? 1 : 0, P.zg,
                       make_double2(P.rp_re, P.rp_im), (double2*)b);
    e = hipGetLastError();
  }
  hipError_t e2 = hipStreamSynchronize(s);  // src is host memory owned by the caller
  hipFreeAsync(d_src, s);
  if (e == hipSuccess) e = e2;
  return to_status(e);
}

extern "C" fmbem_status fmbem_incident_plane_wave(fmbem_plan plan, int32_t n_rhs, const double* dirs,
                                                  double amplitude, void* b, void* hip_stream) {
  return incident(plan, n_rhs, dirs, amplitude, b, hip_stream, 0);
}

extern "C" fmbem_status fmbem_incident_point_source(fmbem_plan plan, int32_t n_rhs, const double* src,
                                                    double amplitude, void* b, void* hip_stream) {
  return incident(plan, n_rhs, src, amplitude, b, hip_stream, 1);
}
