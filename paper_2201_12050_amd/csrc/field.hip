// Post-processing of a solved surface pressure: the pressure at points of the fluid
// and the insertion loss over a set of observation points.
//
// For x in the fluid the solid angle c(x) is 1, and on a rigid surface dp/dn = 0, so
// the CBIE (Sec. 2.1, eq. (cbie)) becomes the representation
//   p(x) = p_inc(x) - int_Gamma dG/dn_y(x, y) p(y) dGamma(y)
//        = p_inc(x) - sum_j p_j W_j(x),   W_j(x) = int_{Delta_j} dG/dn_y(x, y) dA(y),
// with j over the constant elements of every cell of the lattice.  W_j uses the
// non-self Duffy rule of the plan build: q x q points collapsed at the first vertex,
// q = 16 / 8 / 4 for |x - centroid_j| < L_j / < 3 L_j / otherwise.
// The insertion loss (eq. (insertionloss)) is 20 log10(sum_i |p_inc(x_i)| / sum_i |p(x_i)|).
// In the half-space the Green's function carries the image term (Sec. 2.1, eq. (green3dHalf)):
// W_j gains R_p times the weight of the mirrored element, and the incident field its image.
//
// Work split: one workgroup per (point, chunk of kFieldPerThread * 256 elements, group of
// up to kFieldRhs right-hand sides).  Each thread integrates W_j for its elements once and
// applies it to every right-hand side of its group; the workgroup sum goes to a partial
// buffer [R][M][chunks] that a second kernel adds up in chunk order (deterministic).
// The work is FP64 vector arithmetic (sqrt, divide and sincos per quadrature point);
// the element geometry is n x 144 bytes and stays in cache.
#include <cmath>

#include "common.hpp"
#include "geom.hpp"

namespace fmbem {

constexpr int kFieldThreads = 256;
constexpr int kFieldPerThread = 4;
constexpr int kFieldRhs = 4;
constexpr int kFieldChunk = kFieldThreads * kFieldPerThread;

__device__ inline double block_sum256(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();  // red may still be read from the previous call
  if (lane == 0) red[w] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// W_j(x) for the element e of the cell at origin o
__device__ inline double2 dl_weight(const double* x, const Geo& e, const double* o, double k, const QuadTab& Q) {
  double a[3], ba[3], cb[3], ca[3], dc[3];
  for (int t = 0; t < 3; ++t) {
    a[t] = e.a[t] + o[t];
    ba[t] = e.b[t] - e.a[t];
    cb[t] = e.c[t] - e.b[t];
    ca[t] = e.c[t] - e.a[t];
    dc[t] = x[t] - (e.cen[t] + o[t]);
  }
  const double dist = sqrt(dot3(dc, dc));
  const int q = dist < e.longest ? 16 : (dist < 3.0 * e.longest ? 8 : 4);
  const int qo = quad_off(q);
  const double cr[3] = {ba[1] * ca[2] - ba[2] * ca[1], ba[2] * ca[0] - ba[0] * ca[2], ba[0] * ca[1] - ba[1] * ca[0]};
  const double jac = sqrt(dot3(cr, cr));
  double re = 0.0, im = 0.0;
  for (int ia = 0; ia < q; ++ia) {
    const double u = Q.t[qo + ia];
    const double wu = Q.w[qo + ia] * u * jac;
    for (int ib = 0; ib < q; ++ib) {
      const double v = Q.t[qo + ib];
      double r[3];
      for (int t = 0; t < 3; ++t) r[t] = x[t] - (a[t] + u * (ba[t] + v * cb[t]));
      const double2 kv = bm_kernel(r, e.nrm, e.nrm, k, make_double2(0.0, 0.0), false);
      const double wt = wu * Q.w[qo + ib];
      re += wt * kv.x;
      im += wt * kv.y;
    }
  }
  return make_double2(re, im);
}

// the element e of the cell at origin o mirrored in the plane z = zg, vertices (a, c, b) so that
// its normal is the mirrored normal
__device__ inline Geo mirrored(const Geo& e, const double* o, double zg) {
  Geo m;
  for (int t = 0; t < 3; ++t) {
    m.a[t] = e.a[t] + o[t];
    m.b[t] = e.c[t] + o[t];
    m.c[t] = e.b[t] + o[t];
    m.cen[t] = e.cen[t] + o[t];
    m.nrm[t] = e.nrm[t];
  }
  m.a[2] = 2.0 * zg - m.a[2];
  m.b[2] = 2.0 * zg - m.b[2];
  m.c[2] = 2.0 * zg - m.c[2];
  m.cen[2] = 2.0 * zg - m.cen[2];
  m.nrm[2] = -m.nrm[2];
  m.longest = e.longest;
  m.area = e.area;
  return m;
}

// grid: x = point * chunks + chunk, y = group of kFieldRhs right-hand sides.  half != 0 adds
// R_p times the double-layer weight of the mirrored element (half-space Green's function).
__global__ __launch_bounds__(kFieldThreads) void field_kernel(
    const double* __restrict__ geom, int n, int C, int g0, int g1, double p0, double p1, double p2, double k,
    QuadTab Q, const double* __restrict__ pts, int chunks, const double2* __restrict__ xs, int R, int M, int half,
    double zg, double2 rp, double2* __restrict__ part) {
  __shared__ double red[4];
  const int m = blockIdx.x / chunks;
  const int chunk = blockIdx.x - m * chunks;
  const int r0 = blockIdx.y * kFieldRhs;
  const int nr = min(kFieldRhs, R - r0);
  const size_t N = (size_t)n * C;
  const double x[3] = {pts[3 * m], pts[3 * m + 1], pts[3 * m + 2]};
  double2 acc[kFieldRhs];
#pragma unroll
  for (int r = 0; r < kFieldRhs; ++r) acc[r] = make_double2(0.0, 0.0);
  for (int e = 0; e < kFieldPerThread; ++e) {
    const size_t j = (size_t)chunk * kFieldChunk + (size_t)e * kFieldThreads + threadIdx.x;
    if (j >= N) break;
    const int c = (int)(j / n);
    const int i = (int)(j - (size_t)c * n);
    const double o[3] = {(c % g0) * p0, ((c / g0) % g1) * p1, (c / (g0 * g1)) * p2};
    const Geo el = load_geo(geom, i);
    double2 w = dl_weight(x, el, o, k, Q);
    if (half) {
      const double o0[3] = {0.0, 0.0, 0.0};
      w = cadd<double>(w, cmul<double>(rp, dl_weight(x, mirrored(el, o, zg), o0, k, Q)));
    }
#pragma unroll
    for (int r = 0; r < kFieldRhs; ++r)
      if (r < nr) cfma<double>(acc[r], w, xs[(size_t)(r0 + r) * N + j]);
  }
#pragma unroll
  for (int r = 0; r < kFieldRhs; ++r) {
    if (r >= nr) break;  // uniform over the workgroup
    const double sx = block_sum256(acc[r].x, red);
    const double sy = block_sum256(acc[r].y, red);
    if (threadIdx.x == 0) part[((size_t)(r0 + r) * M + m) * chunks + chunk] = make_double2(sx, sy);
  }
}

// p[r][m] = p_inc[r][m] - sum over chunks (p may alias p_inc)
__global__ void field_finish_kernel(const double2* __restrict__ part, int chunks, int RM, const double2* p_inc,
                                    double2* p) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= RM) return;
  const double2* q = part + (size_t)idx * chunks;
  double sx = 0.0, sy = 0.0;
  for (int c = 0; c < chunks; ++c) {
    sx += q[c].x;
    sy += q[c].y;
  }
  double2 v = p_inc ? p_inc[idx] : make_double2(0.0, 0.0);
  v.x -= sx;
  v.y -= sy;
  p[idx] = v;
}

// incident pressure at arbitrary points: plane wave A e^{ik d.x} (Sec. 4.1, eq. (planewave))
// or monopole A e^{ikR}/R (Sec. 4.2); out [R][M]
// (half != 0: plus R_p times the incident field at the mirrored point, the image of the field)
__device__ inline double2 incident_value(const double* x, const double* s, int point, double k, double amp) {
  double ph, mag;
  if (!point) {
    ph = k * dot3(s, x);
    mag = amp;
  } else {
    const double d[3] = {x[0] - s[0], x[1] - s[1], x[2] - s[2]};
    const double Rd = sqrt(dot3(d, d));
    ph = k * Rd;
    mag = amp / Rd;
  }
  double sn, cs;
  sincos(ph, &sn, &cs);
  return make_double2(mag * cs, mag * sn);
}

__global__ void incident_points_kernel(double k, int R, const double* __restrict__ src, int point, double amp,
                                       const double* __restrict__ pts, int M, int half, double zg, double2 rp,
                                       double2* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= R * M) return;
  const int r = idx / M, m = idx - r * M;
  const double* s = src + 3 * r;
  const double* x = pts + 3 * m;
  double2 v = incident_value(x, s, point, k, amp);
  if (half) {
    const double xm[3] = {x[0], x[1], 2.0 * zg - x[2]};
    v = cadd<double>(v, cmul<double>(rp, incident_value(xm, s, point, k, amp)));
  }
  out[idx] = v;
}

// il[r] = 20 log10(sum_m |p_inc[r][m]| / sum_m |p[r][m]|), one workgroup per right-hand side
__global__ __launch_bounds__(256) void insertion_loss_kernel(const double2* __restrict__ p_inc,
                                                             const double2* __restrict__ p, int M,
                                                             double* __restrict__ il) {
  __shared__ double red[4];
  const size_t base = (size_t)blockIdx.x * M;
  double a = 0.0, b = 0.0;
  for (int m = threadIdx.x; m < M; m += 256) {
    const double2 u = p_inc[base + m], v = p[base + m];
    a += hypot(u.x, u.y);
    b += hypot(v.x, v.y);
  }
  a = block_sum256(a, red);
  b = block_sum256(b, red);
  if (threadIdx.x == 0) il[blockIdx.x] = 20.0 * log10(a / b);
}

// copy host points to the device (stream-ordered); caller frees with hipFreeAsync
static hipError_t upload_points(const double* host, int count, double** dev, hipStream_t s) {
  *dev = nullptr;
  hipError_t e = hipMallocAsync((void**)dev, (size_t)3 * count * sizeof(double), s);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(*dev, host, (size_t)3 * count * sizeof(double), hipMemcpyHostToDevice, s);
}

static bool all_finite(const double* v, size_t count) {
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

}  // namespace fmbem

using namespace fmbem;

extern "C" fmbem_status fmbem_incident_at_points(fmbem_plan plan, int32_t kind, int32_t n_rhs, const double* src,
                                                 double amplitude, int32_t n_points, const double* points,
                                                 void* p_inc, void* hip_stream) {
  if (!plan || !src || !points || !p_inc || n_rhs < 1 || n_points < 1 || (kind != 0 && kind != 1) ||
      !std::isfinite(amplitude))
    return FMBEM_ERR_INVALID_ARG;
  if ((int64_t)n_rhs * n_points > INT32_MAX) return FMBEM_ERR_UNSUPPORTED;
  if (!all_finite(src, (size_t)3 * n_rhs) || !all_finite(points, (size_t)3 * n_points)) return FMBEM_ERR_INVALID_ARG;
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  double *d_src = nullptr, *d_pts = nullptr;
  hipError_t e = upload_points(src, n_rhs, &d_src, s);
  if (e == hipSuccess) e = upload_points(points, n_points, &d_pts, s);
  if (e == hipSuccess) {
    const int total = n_rhs * n_points;
    hipLaunchKernelGGL(incident_points_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, P.k, n_rhs,
                       d_src, kind, amplitude, d_pts, n_points, P.half ? 1 : 0, P.zg, make_double2(P.rp_re, P.rp_im),
                       (double2*)p_inc);
    e = hipGetLastError();
  }
  const hipError_t e2 = hipStreamSynchronize(s);  // src and points are host memory owned by the caller
  if (d_src) hipFreeAsync(d_src, s);
  if (d_pts) hipFreeAsync(d_pts, s);
  if (e == hipSuccess) e = e2;
  return to_status(e);
}

extern "C" fmbem_status fmbem_field(fmbem_plan plan, int32_t n_rhs, const void* x, int32_t n_points,
                                    const double* points, const void* p_inc, void* p, void* hip_stream) {
  if (!plan || !x || !points || !p || n_rhs < 1 || n_points < 1) return FMBEM_ERR_INVALID_ARG;
  if (!all_finite(points, (size_t)3 * n_points)) return FMBEM_ERR_INVALID_ARG;
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  const size_t N = (size_t)P.n * P.C;
  const size_t chunks = (N + kFieldChunk - 1) / kFieldChunk;
  const size_t groups = ((size_t)n_rhs + kFieldRhs - 1) / kFieldRhs;
  if ((int64_t)n_rhs * n_points > INT32_MAX || chunks * (size_t)n_points > (size_t)INT32_MAX || groups > 65535)
    return FMBEM_ERR_UNSUPPORTED;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  double* d_pts = nullptr;
  double2* part = nullptr;
  hipError_t e = upload_points(points, n_points, &d_pts, s);
  if (e == hipSuccess)
    e = hipMallocAsync((void**)&part, (size_t)n_rhs * n_points * chunks * sizeof(double2), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(field_kernel, dim3((unsigned)(chunks * n_points), (unsigned)groups), dim3(kFieldThreads), 0,
                       s, P.geom, P.n, P.C, P.grid[0], P.grid[1], P.pitch[0], P.pitch[1], P.pitch[2], P.k, P.quad,
                       d_pts, (int)chunks, (const double2*)x, n_rhs, n_points, P.half ? 1 : 0, P.zg,
                       make_double2(P.rp_re, P.rp_im), part);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const int RM = n_rhs * n_points;
    hipLaunchKernelGGL(field_finish_kernel, dim3((unsigned)((RM + 255) / 256)), dim3(256), 0, s, part, (int)chunks,
                       RM, (const double2*)p_inc, (double2*)p);
    e = hipGetLastError();
  }
  const hipError_t e2 = hipStreamSynchronize(s);  // points are host memory owned by the caller
  if (d_pts) hipFreeAsync(d_pts, s);
  if (part) hipFreeAsync(part, s);
  if (e == hipSuccess) e = e2;
  return to_status(e);
}

extern "C" fmbem_status fmbem_insertion_loss(int32_t n_rhs, int32_t n_points, const void* p_inc, const void* p,
                                             double* il, void* hip_stream) {
  if (!p_inc || !p || !il || n_rhs < 1 || n_points < 1) return FMBEM_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(insertion_loss_kernel, dim3((unsigned)n_rhs), dim3(256), 0, s, (const double2*)p_inc,
                     (const double2*)p, n_points, il);
  return to_status(hipGetLastError());
}
