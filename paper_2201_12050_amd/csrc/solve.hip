// Restarted GMRES with FP64 Arnoldi (classical Gram-Schmidt with the DGKS selective
// second pass), Givens rotations and FP64 iterative refinement around FP32 inner solves.
//
// The paper solves the FMPBEM system iteratively with GMRES (Sec. 2.4, Sec. 3.5,
// Sec. 4).  All right-hand sides are iterated together, each in its own Krylov
// space; vectors are [R][N] complex128.  Per Arnoldi step:
//   w = A v_j, built in the slot of v_{j+1}   (operator in FP64, or FP32 with FP64 output)
//   h = V^H w, w -= V h                       (multi-dot and multi-axpy kernels, FP64)
//   if ||w_new|| < ||w_old|| / sqrt(2): h2 = V^H w, w -= V h2, h += h2   (device-side decision)
//   h_{j+1} = ||w||, v_{j+1} = w / h_{j+1}
//   Givens update of the Hessenberg column and of g on the device (one workgroup per RHS)
// The host learns the residual estimates |g_{j+1}| one step late: step j+1 is
// already queued when it waits for step j, so the device never idles on the
// host; a step queued after convergence is discarded by the per-RHS freeze.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <cstdint>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace fmbem {

constexpr int kDotThreads = 256;
constexpr int kDotEl = 4;    // elements per thread in the multi-dot kernel
constexpr int kDotVec = 8;   // basis vectors per workgroup

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// part[r][i][blk] = sum_{n in block} conj(V_i[r][n]) w[r][n]; workgroup (bx, by, r) of a grid
// (nblk blocks, vector groups of 8, R)
__device__ __attribute__((always_inline)) inline void mdot_body(const double2* __restrict__ V, size_t vstride, const double2* __restrict__ w,
                                 size_t N, int J, double2* __restrict__ part, const int* __restrict__ flag, int bx,
                                 int by, int r, int nblk) {
  __shared__ double2 red[kDotThreads / 64][kDotVec];
  if (flag && !flag[r]) return;  // conditional pass not needed for this RHS
  const int i0 = by * kDotVec;
  const size_t base = (size_t)bx * kDotThreads * kDotEl + threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // every load first, from clamped indices (an element past N has w = 0, a vector past J is
  // never written out), so that all kDotVec x kDotEl loads are in flight together
  double2 wl[kDotEl];
  size_t nc[kDotEl];
#pragma unroll
  for (int e = 0; e < kDotEl; ++e) {
    const size_t n = base + (size_t)e * kDotThreads;
    nc[e] = n < N ? n : N - 1;
    wl[e] = w[(size_t)r * N + nc[e]];
    if (n >= N) wl[e] = make_double2(0, 0);
  }
  double2 a[kDotVec][kDotEl];
#pragma unroll
  for (int q = 0; q < kDotVec; ++q) {
    const double2* vi = V + (size_t)min(i0 + q, J - 1) * vstride + (size_t)r * N;
#pragma unroll
    for (int e = 0; e < kDotEl; ++e) a[q][e] = vi[nc[e]];
  }
  double2 acc[kDotVec];
#pragma unroll
  for (int q = 0; q < kDotVec; ++q) {
    acc[q] = make_double2(0, 0);
#pragma unroll
    for (int e = 0; e < kDotEl; ++e) {
      acc[q].x += a[q][e].x * wl[e].x + a[q][e].y * wl[e].y;
      acc[q].y += a[q][e].x * wl[e].y - a[q][e].y * wl[e].x;
    }
  }
#pragma unroll
  for (int q = 0; q < kDotVec; ++q) {
    const double sx = wave_sum(acc[q].x), sy = wave_sum(acc[q].y);
    if (lane == 0) red[wv][q] = make_double2(sx, sy);
  }
  __syncthreads();
  if (threadIdx.x < kDotVec && i0 + (int)threadIdx.x < J) {
    double2 s = red[0][threadIdx.x];
    for (int t = 1; t < kDotThreads / 64; ++t) {
      s.x += red[t][threadIdx.x].x;
      s.y += red[t][threadIdx.x].y;
    }
    part[((size_t)r * J + i0 + threadIdx.x) * nblk + bx] = s;
  }
}

__global__ __launch_bounds__(kDotThreads) void mdot_kernel(const double2* __restrict__ V, size_t vstride,
                                                           const double2* __restrict__ w, size_t N, int J,
                                                           double2* __restrict__ part, const int* __restrict__ flag) {
  mdot_body(V, vstride, w, N, J, part, flag, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x);
}

// one wave per (r, i) sums the block partials s; mode 0: h = s; mode 2: h = sqrt(Re s);
// mode 3: h2 = s and h += s (second Gram-Schmidt pass)
__device__ __attribute__((always_inline)) inline void finish_body(const double2* __restrict__ part, int nblk, int R, int J, double2* __restrict__ h,
                                   int hstride, int mode, double2* __restrict__ h2, const int* __restrict__ flag,
                                   int bx) {
  const int t = bx * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= R * J) return;
  const int r = t / J, i = t - r * J;
  if (flag && !flag[r]) return;
  double sx = 0.0, sy = 0.0;
  for (int b = lane; b < nblk; b += 64) {
    const double2 v = part[(size_t)t * nblk + b];
    sx += v.x;
    sy += v.y;
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  if (lane != 0) return;
  double2* o = h + (size_t)r * hstride + i;
  if (mode == 0) *o = make_double2(sx, sy);
  else if (mode == 2) *o = make_double2(isnan(sx) ? sx : sqrt(fmax(sx, 0.0)), 0.0);  // NaN stays visible
  else {
    h2[(size_t)r * hstride + i] = make_double2(sx, sy);
    o->x += sx;
    o->y += sy;
  }
}

__global__ void mdot_finish(const double2* __restrict__ part, int nblk, int R, int J, double2* __restrict__ h,
                            int hstride, int mode, double2* __restrict__ h2, const int* __restrict__ flag) {
  finish_body(part, nblk, R, J, h, hstride, mode, h2, flag, blockIdx.x);
}

// w[r][n] += sgn * sum_{i<J} c[r][i] V_i[r][n]; with npart, also per-block sums of |w|^2
__device__ __attribute__((always_inline)) inline void maxpy_body(const double2* __restrict__ V, size_t vstride, const double2* __restrict__ c,
                                  int cstride, double2* __restrict__ w, size_t N, int J, double sgn,
                                  double* __restrict__ npart, const int* __restrict__ flag, int bx, int r, int gx) {
  extern __shared__ double2 cs[];
  __shared__ double red[4];
  if (flag && !flag[r]) return;
  for (int i = threadIdx.x; i < J; i += blockDim.x) cs[i] = c[(size_t)r * cstride + i];
  __syncthreads();
  double nn = 0.0;
  for (size_t n = (size_t)bx * blockDim.x + threadIdx.x; n < N; n += (size_t)gx * blockDim.x) {
    double2 acc = w[(size_t)r * N + n];
    for (int i = 0; i < J; ++i) {
      const double2 v = V[i * vstride + (size_t)r * N + n];
      acc.x += sgn * (cs[i].x * v.x - cs[i].y * v.y);
      acc.y += sgn * (cs[i].x * v.y + cs[i].y * v.x);
    }
    w[(size_t)r * N + n] = acc;
    nn += acc.x * acc.x + acc.y * acc.y;
  }
  if (npart) {
    nn = wave_sum(nn);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nn;
    __syncthreads();
    if (threadIdx.x == 0) npart[(size_t)r * gx + bx] = red[0] + red[1] + red[2] + red[3];
  }
}

__global__ __launch_bounds__(256) void maxpy_kernel(const double2* __restrict__ V, size_t vstride,
                                                    const double2* __restrict__ c, int cstride,
                                                    double2* __restrict__ w, size_t N, int J, double sgn,
                                                    double* __restrict__ npart, const int* __restrict__ flag) {
  maxpy_body(V, vstride, c, cstride, w, N, J, sgn, npart, flag, blockIdx.x, blockIdx.y, gridDim.x);
}

// DGKS criterion (Daniel, Gragg, Kaufman & Stewart, 1976): a second Gram-Schmidt pass is
// needed when the projection removed more than 1 - 1/sqrt(2) of the norm, i.e. when
// ||w'|| < ||w|| / sqrt(2).  ||w||^2 is the last dot of the first pass (hc[j+1]);
// ||w'||^2 is the sum of the first multi-axpy's partials.  One workgroup per RHS.
// mode: 0 DGKS, 1 always, 2 never.
__global__ __launch_bounds__(256) void reorth_check_kernel(int mode, int nb, const double* __restrict__ npart,
                                                           const double2* __restrict__ hc, int hstride, int j,
                                                           const int* __restrict__ jdone, int* __restrict__ flag) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += npart[(size_t)r * nb + b];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double w2 = hc[(size_t)r * hstride + j + 1].x;
    const bool need = mode == 1 || (mode == 0 && 2.0 * (red[0] + red[1] + red[2] + red[3]) < w2);
    flag[r] = (jdone[r] < 0 && need) ? 1 : 0;
  }
}

// out[r][n] = a[r][n] / s[r] (s = .x of a double2 array; 0 when s = 0); optional FP32 copy; may run in place
__global__ void scale_kernel(const double2* a, const double2* __restrict__ s, int sstride, double2* out,
                             float2* __restrict__ out32, size_t N) {
  const int r = blockIdx.y;
  const double d = s[(size_t)r * sstride].x;
  const double f = d > 0 ? 1.0 / d : 0.0;
  for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (size_t)gridDim.x * blockDim.x) {
    const double2 v = a[(size_t)r * N + n];
    const double2 o = make_double2(v.x * f, v.y * f);
    out[(size_t)r * N + n] = o;
    if (out32) out32[(size_t)r * N + n] = make_float2((float)o.x, (float)o.y);
  }
}

// out = a - b
__global__ void sub_kernel(const double2* __restrict__ a, const double2* __restrict__ b, double2* __restrict__ out,
                           size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = make_double2(a[i].x - b[i].x, a[i].y - b[i].y);
}

__global__ void add_kernel(double2* __restrict__ a, const double2* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    a[i] = make_double2(a[i].x + b[i].x, a[i].y + b[i].y);
}

__global__ void zero_kernel(double2* __restrict__ a, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    a[i] = make_double2(0, 0);
}

__global__ void copy_kernel(double2* __restrict__ a, const double2* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) a[i] = b[i];
}

__global__ void to32_kernel(const double2* __restrict__ a, float2* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

__global__ void to64_kernel(const float2* __restrict__ a, double2* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = make_double2((double)a[i].x, (double)a[i].y);
}

// sqrt of the sum of RHS r's nb |w|^2 block partials, the same fixed order in every workgroup
__device__ inline double partial_norm(const double* __restrict__ npart, int nb, int r) {
  __shared__ double red[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += npart[(size_t)r * nb + b];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  return sqrt(fmax(red[0] + red[1] + red[2] + red[3], 0.0));
}

// Arnoldi step close: v_{j+1} = w / ||w|| (and its FP32 copy), ||w|| from the multi-axpy's
// partials, recomputed by every workgroup.  Workgroup (0, r) also writes hn and does the
// Givens update of Hessenberg column j (rotations [[conj(c), conj(s)], [-s, c]]) and of g on
// LDS copies, the residual estimate |g_{j+1}| and the freeze flag (also written to mapped
// host memory for the host's convergence check).  Grid (blocks, R), 256 threads.
constexpr int kMaxRestart = 1000;
__device__ __attribute__((always_inline)) inline void scale_givens_body(const double* __restrict__ npart, int nb, int m, int j,
                                         const double2* __restrict__ hc, int hstride, double2* __restrict__ hn,
                                         double2* __restrict__ H, double2* __restrict__ cs, double2* __restrict__ sn,
                                         double2* __restrict__ g, double* __restrict__ res, int* __restrict__ jdone,
                                         int* __restrict__ jdone_host, const double* __restrict__ tol,
                                         double2* __restrict__ w, float2* __restrict__ w32, size_t N, int bx, int r,
                                         int gx) {
  const double nrm = partial_norm(npart, nb, r);
  const double f = nrm > 0 ? 1.0 / nrm : 0.0;
  for (size_t n = (size_t)bx * blockDim.x + threadIdx.x; n < N; n += (size_t)gx * blockDim.x) {
    const double2 v = w[(size_t)r * N + n];
    const double2 o = make_double2(v.x * f, v.y * f);
    w[(size_t)r * N + n] = o;
    if (w32) w32[(size_t)r * N + n] = make_float2((float)o.x, (float)o.y);
  }
  if (bx != 0) return;
  // LDS (dynamic, 3m + 2 entries): Hessenberg column, cosines and sines of the earlier rotations
  extern __shared__ double2 gv_lds[];
  double2* col = gv_lds;
  double2* lc = col + m + 2;
  double2* ls = lc + m;
  const int frozen = jdone[r];
  if (threadIdx.x == 0) hn[(size_t)r * hstride] = make_double2(nrm, 0.0);
  if (frozen >= 0) {
    if (threadIdx.x == 0) jdone_host[r] = frozen;
    return;
  }
  double2* Hr = H + (size_t)r * (m + 1) * m;
  double2* c = cs + (size_t)r * m;
  double2* sg = sn + (size_t)r * m;
  double2* gr = g + (size_t)r * (m + 1);
  for (int i = threadIdx.x; i <= j; i += blockDim.x) col[i] = hc[(size_t)r * hstride + i];
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    lc[i] = c[i];
    ls[i] = sg[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    col[j + 1] = make_double2(nrm, 0.0);
    for (int i = 0; i < j; ++i) {
      const double2 a = col[i], b = col[i + 1];
      col[i] = cadd<double>(cmul<double>(cconj<double>(lc[i]), a), cmul<double>(cconj<double>(ls[i]), b));
      col[i + 1] = csub<double>(cmul<double>(lc[i], b), cmul<double>(ls[i], a));
    }
    const double2 a = col[j], b = col[j + 1];
    const double den = sqrt(a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y);
    double2 cj = make_double2(1, 0), sj = make_double2(0, 0);
    if (den > 0) {
      cj = make_double2(a.x / den, a.y / den);
      sj = make_double2(b.x / den, b.y / den);
    }
    c[j] = cj;
    sg[j] = sj;
    col[j] = make_double2(den, 0.0);
    col[j + 1] = make_double2(0, 0);
    const double2 gj = gr[j];
    const double2 g1 = csub<double>(make_double2(0, 0), cmul<double>(sj, gj));
    gr[j + 1] = g1;
    gr[j] = cmul<double>(cconj<double>(cj), gj);
    const double e = sqrt(g1.x * g1.x + g1.y * g1.y);
    res[r] = e;
    const int jd = (e <= tol[r] || den == 0.0 || nrm == 0.0) ? j + 1 : -1;
    jdone[r] = jd;
    jdone_host[r] = jd;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) Hr[(size_t)i * m + j] = col[i];
}

__global__ __launch_bounds__(256) void scale_givens_kernel(const double* __restrict__ npart, int nb, int m, int j,
                                                           const double2* __restrict__ hc, int hstride,
                                                           double2* __restrict__ hn, double2* __restrict__ H,
                                                           double2* __restrict__ cs, double2* __restrict__ sn,
                                                           double2* __restrict__ g, double* __restrict__ res,
                                                           int* __restrict__ jdone, int* __restrict__ jdone_host,
                                                           const double* __restrict__ tol, double2* __restrict__ w,
                                                           float2* __restrict__ w32, size_t N) {
  scale_givens_body(npart, nb, m, j, hc, hstride, hn, H, cs, sn, g, res, jdone, jdone_host, tol, w, w32, N,
                    blockIdx.x, blockIdx.y, gridDim.x);
}

// y = H^{-1} g (upper triangular, size jdone[r] or jcur) by column sweeps; one workgroup per RHS
__global__ __launch_bounds__(256) void backsolve_kernel(int m, int jcur, const double2* __restrict__ H,
                                                        const double2* __restrict__ g,
                                                        const int* __restrict__ jdone, double2* __restrict__ y,
                                                        int ystride) {
  extern __shared__ double2 gl[];  // [m + 1]
  __shared__ double2 yi;
  const int r = blockIdx.x;
  const int J = jdone[r] >= 0 ? jdone[r] : jcur;
  const double2* Hr = H + (size_t)r * (m + 1) * m;
  double2* yr = y + (size_t)r * ystride;
  for (int i = threadIdx.x; i < J; i += blockDim.x) gl[i] = g[(size_t)r * (m + 1) + i];
  for (int i = J + threadIdx.x; i < ystride; i += blockDim.x) yr[i] = make_double2(0, 0);
  __syncthreads();
  for (int i = J - 1; i >= 0; --i) {
    if (threadIdx.x == 0) {
      const double2 d = Hr[(size_t)i * m + i];
      const double dd = d.x * d.x + d.y * d.y;
      const double2 acc = gl[i];
      yi = dd > 0 ? make_double2((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd)
                  : make_double2(0, 0);
      yr[i] = yi;
    }
    __syncthreads();
    const double2 v = yi;
    for (int t = threadIdx.x; t < i; t += blockDim.x) gl[t] = csub<double>(gl[t], cmul<double>(Hr[(size_t)t * m + i], v));
    __syncthreads();
  }
}

// out[r] = hn[r * hstride].x (residual norms into mapped host memory)
__global__ void norm_out_kernel(const double2* __restrict__ hn, int hstride, int R, double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < R) out[r] = hn[(size_t)r * hstride].x;
}

// g = [beta, 0, ...], jdone = -1 (beta from the .x of hn); beta <= tol freezes at 0
__global__ void gmres_init_kernel(int R, int m, const double2* __restrict__ beta, int hstride,
                                  const double* __restrict__ tol, double2* __restrict__ g, int* __restrict__ jdone,
                                  int* __restrict__ jdone_host, double* __restrict__ res) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const double b = beta[(size_t)r * hstride].x;
  for (int i = 0; i <= m; ++i) g[(size_t)r * (m + 1) + i] = make_double2(0, 0);
  g[(size_t)r * (m + 1)] = make_double2(b, 0);
  jdone[r] = b > tol[r] ? -1 : 0;
  jdone_host[r] = jdone[r];
  res[r] = b;
}

// Classical Gram-Schmidt of several members' Arnoldi steps in shared launches: each of the four
// kernels of a single-pass step (dots, their reduction, the multi-axpy with |w|^2 partials, the
// normalisation with the Givens update) runs once for all members of a round.  Member q owns the
// workgroups [block0[q], block0[q+1]) of a launch and sees the same local workgroup indices and
// grid sizes as its own launch would give it, so its results are bitwise those of the
// per-member sequence.
struct GsDev {  // a member's buffers and sizes, copied to the device when the member is set up
  double2 *V, *part, *hc, *hn, *H, *cs, *sn, *g;
  double *res, *tolv, *npart;
  int* jdone;
  int* djd[2];
  float2* x32;
  size_t N, vlen;
  int R, nblk, nb, hstride, m;
};
constexpr int kMaxGsJobs = 32;
struct GsJobs {
  int count;
  const GsDev* d[kMaxGsJobs];
  int j[kMaxGsJobs];     // Arnoldi step: w = A v_j sits in the slot of v_{j+1}
  int mode[kMaxGsJobs];  // bit 0: round slot of the freeze flags, bit 1: FP32 copy of v_{j+1}
  int block0[kMaxGsJobs + 1];
};
__device__ inline int gs_job(const GsJobs& J) {
  int q = 0;
  while (q + 1 < J.count && (int)blockIdx.x >= J.block0[q + 1]) ++q;
  return q;
}
// workgroups of member q in each kernel
static inline int gs_blocks(int kernel, const GsDev& h, int j) {
  if (kernel == 0) return h.nblk * ((j + 2 + kDotVec - 1) / kDotVec) * h.R;
  if (kernel == 1) return (h.R * (j + 2) + 3) / 4;
  return h.nb * h.R;
}

__global__ __launch_bounds__(kDotThreads) void gs_mdot_kernel(GsJobs J) {
  const int q = gs_job(J);
  const GsDev& D = *J.d[q];
  const int jn = J.j[q] + 2, ny = (jn + kDotVec - 1) / kDotVec;
  const int l = (int)blockIdx.x - J.block0[q];
  const int bx = l % D.nblk, by = (l / D.nblk) % ny, r = l / (D.nblk * ny);
  mdot_body(D.V, D.vlen, D.V + (size_t)(J.j[q] + 1) * D.vlen, D.N, jn, D.part, nullptr, bx, by, r, D.nblk);
}
__global__ void gs_finish_kernel(GsJobs J) {
  const int q = gs_job(J);
  const GsDev& D = *J.d[q];
  finish_body(D.part, D.nblk, D.R, J.j[q] + 2, D.hc, D.hstride, 0, nullptr, nullptr, (int)blockIdx.x - J.block0[q]);
}
__global__ __launch_bounds__(256) void gs_maxpy_kernel(GsJobs J) {
  const int q = gs_job(J);
  const GsDev& D = *J.d[q];
  const int l = (int)blockIdx.x - J.block0[q];
  maxpy_body(D.V, D.vlen, D.hc, D.hstride, D.V + (size_t)(J.j[q] + 1) * D.vlen, D.N, J.j[q] + 1, -1.0, D.npart,
             nullptr, l % D.nb, l / D.nb, D.nb);
}
__global__ __launch_bounds__(256) void gs_scale_givens_kernel(GsJobs J) {
  const int q = gs_job(J);
  const GsDev& D = *J.d[q];
  const int l = (int)blockIdx.x - J.block0[q], md = J.mode[q];
  scale_givens_body(D.npart, D.nb, D.m, J.j[q], D.hc, D.hstride, D.hn, D.H, D.cs, D.sn, D.g, D.res, D.jdone,
                    D.djd[md & 1], D.tolv, D.V + (size_t)(J.j[q] + 1) * D.vlen, (md & 2) ? D.x32 : nullptr, D.N,
                    l % D.nb, l / D.nb, D.nb);
}

// One linear system set (a plan and R right-hand sides) advanced one operator application
// per round.  A round of a group: pre() of every member (kernels that precede the
// application and the application request), the group's applications (one grouped launch
// sequence per precision), post() of every member (Gram-Schmidt, Givens, residuals), an
// event; then the host reads the previous round's results (process()) while this round
// runs.  Arnoldi steps continue speculatively on the one-round-late convergence flags (a
// step queued after convergence is frozen on the device and discarded); true residuals
// make the member wait one round for the host's decision.
// Pinned host buffers of finished problems, kept for reuse: freeing pinned memory
// synchronises the device, which would stall the rounds of every other problem in flight.
static std::mutex g_pin_mu;
static std::multimap<std::pair<size_t, unsigned>, void*> g_pin_free;
static size_t pin_bytes(size_t b) { return (b + 255) / 256 * 256; }
static hipError_t pinned_get(void** p, size_t bytes, unsigned flags) {
  bytes = pin_bytes(bytes);
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    auto it = g_pin_free.find({bytes, flags});
    if (it != g_pin_free.end()) {
      *p = it->second;
      g_pin_free.erase(it);
      return hipSuccess;
    }
  }
  return hipHostMalloc(p, bytes, flags);
}
static void pinned_put(void* p, size_t bytes, unsigned flags) {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free.insert({{pin_bytes(bytes), flags}, p});
}
constexpr unsigned kMapped = hipHostMallocMapped | hipHostMallocCoherent;

struct Member {
  const Plan& P;
  hipStream_t s;
  int R, m;
  int ortho = 0;   // FMBEM_ORTHO_*
  int ip = 0;      // inner precision
  double tol = 0, inner_tol = 0;
  int max_its = 0, max_ref = 0;
  const double2* b = nullptr;
  double2* x = nullptr;
  size_t N;        // DOFs per RHS
  size_t vlen;     // R * N
  int nblk;
  int hstride;
  int nb;          // workgroups of the multi-axpy kernel (and of its norm partials)
  std::vector<void*> mem;
  hipMemPool_t pool = nullptr;  // set: device buffers are stream-ordered allocations from this pool
  double2 *V = nullptr, *r = nullptr, *d = nullptr, *t = nullptr, *rin = nullptr;
  float2* x32 = nullptr;
  void* ws = nullptr;
  double2 *part = nullptr, *hc = nullptr, *hn = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr,
          *y = nullptr;
  double *res = nullptr, *tolv = nullptr, *npart = nullptr;
  int* jdone = nullptr;
  int* reorth = nullptr;  // per-RHS second Gram-Schmidt pass flag
  // per round slot: freeze flags and residual norms written by the device into mapped host memory
  int* hjd[2] = {nullptr, nullptr};
  int* djd[2] = {nullptr, nullptr};
  double* hres[2] = {nullptr, nullptr};
  double* dres[2] = {nullptr, nullptr};
  double* htol = nullptr;  // pinned staging of per-RHS tolerances
  GsDev gsh{};             // host image of gsd (kept: the copy to the device is asynchronous)
  GsDev* gsd = nullptr;    // this member's buffers for the grouped Gram-Schmidt kernels

  // state
  enum Phase { RUN_TRUE, START_INNER, RUN_RESTART, RUN_ARN, CLOSE, WAIT, DONE };
  enum Kind { K_NONE, K_INIT, K_TRUE, K_RESTART, K_ARN };
  struct Rec {
    int kind = K_NONE, j = 0, epoch = 0;
  };
  Rec rec[2];
  int phase = RUN_TRUE;
  int after_close = RUN_TRUE;
  int gm_prec = 0;                 // precision of the current GMRES
  const double2* gm_rhs = nullptr;
  double2* gm_sol = nullptr;
  int j = 0;                       // Arnoldi steps queued in the current cycle
  int epoch = 0;
  int its = 0, refs = 0;
  bool x_zero = false;  // every RHS starts from x = 0 (set by started(), cleared by the first true residual)
  bool ok = false;
  bool bad_input = false;
  bool emit = true;  // false: post() updates host state only (a captured graph replays the kernels)
  hipError_t err = hipSuccess;
  std::vector<double> bn, rel;
  // this round's application
  bool req = false;
  int req_prec = 0;
  const void* req_in = nullptr;
  double2* req_out = nullptr;

  Member(const Plan& p_, hipStream_t s_, int R_, int m_) : P(p_), s(s_), R(R_), m(m_) {
    N = (size_t)P.n * P.C;
    vlen = (size_t)R * N;
    nblk = (int)((N + kDotThreads * kDotEl - 1) / (kDotThreads * kDotEl));
    hstride = m + 2;
    // multi-axpy workgroups: each step-closing workgroup re-sums their |w|^2 partials
    nb = (int)std::min<size_t>((N + 255) / 256, 512);
    bn.assign(R, 0.0);
    rel.assign(R, 0.0);
  }
  ~Member() {
    for (void* q : mem) {
      if (pool)
        hipFreeAsync(q, s);  // after the member's last work on its stream
      else
        hipFree(q);
    }
    for (int i = 0; i < 2; ++i) {
      if (hjd[i]) pinned_put(hjd[i], R * sizeof(int), kMapped);
      if (hres[i]) pinned_put(hres[i], 2 * R * sizeof(double), kMapped);
    }
    if (htol) pinned_put(htol, R * sizeof(double), hipHostMallocDefault);
  }
  // device buffers of a member, in allocation order (footprint() sums exactly these)
  struct Buf {
    void** ptr;
    size_t bytes;
  };
  std::vector<Buf> buffers(bool need32) {
    const size_t wsb = (size_t)R * std::max(matvec_workspace_bytes_per_rhs(P, 0),
                                            need32 ? matvec_workspace_bytes_per_rhs(P, 1) : 0);
    std::vector<Buf> v{{(void**)&V, (size_t)(m + 1) * vlen * sizeof(double2)},
                       {(void**)&r, vlen * sizeof(double2)},
                       {(void**)&d, vlen * sizeof(double2)},
                       {(void**)&t, vlen * sizeof(double2)},
                       {(void**)&rin, vlen * sizeof(double2)},
                       {&ws, wsb},
                       {(void**)&part, (size_t)R * (m + 1) * nblk * sizeof(double2)},
                       {(void**)&hc, (size_t)R * hstride * sizeof(double2)},
                       {(void**)&hn, (size_t)R * hstride * sizeof(double2)},
                       {(void**)&H, (size_t)R * (m + 1) * m * sizeof(double2)},
                       {(void**)&cs, (size_t)R * m * sizeof(double2)},
                       {(void**)&sn, (size_t)R * m * sizeof(double2)},
                       {(void**)&g, (size_t)R * (m + 1) * sizeof(double2)},
                       {(void**)&y, (size_t)R * hstride * sizeof(double2)},
                       {(void**)&res, R * sizeof(double)},
                       {(void**)&tolv, R * sizeof(double)},
                       {(void**)&jdone, R * sizeof(int)},
                       {(void**)&npart, (size_t)R * nb * sizeof(double)},
                       {(void**)&reorth, R * sizeof(int)},
                       {(void**)&gsd, sizeof(GsDev)}};
    if (need32) v.push_back({(void**)&x32, vlen * sizeof(float2)});
    for (Buf& q : v) q.bytes = std::max<size_t>((q.bytes + 255) / 256 * 256, 256);
    return v;
  }
  // device bytes this member allocates (the serving engine's admission unit)
  size_t footprint(bool need32) {
    size_t sum = 0;
    for (const Buf& q : buffers(need32)) sum += q.bytes;
    return sum;
  }
  hipError_t setup(bool need32, hipMemPool_t from = nullptr) {
    hipError_t e;
    pool = from;
    for (const Buf& q : buffers(need32)) {
      if ((e = pool ? hipMallocFromPoolAsync(q.ptr, q.bytes, pool, s) : hipMalloc(q.ptr, q.bytes))) return e;
      mem.push_back(*q.ptr);
    }
    for (int i = 0; i < 2; ++i) {
      if ((e = pinned_get((void**)&hjd[i], R * sizeof(int), kMapped))) return e;
      if ((e = hipHostGetDevicePointer((void**)&djd[i], hjd[i], 0))) return e;
      if ((e = pinned_get((void**)&hres[i], 2 * R * sizeof(double), kMapped))) return e;
      if ((e = hipHostGetDevicePointer((void**)&dres[i], hres[i], 0))) return e;
    }
    if ((e = pinned_get((void**)&htol, R * sizeof(double), hipHostMallocDefault))) return e;
    gsh = GsDev{V, part, hc, hn, H, cs, sn, g, res, tolv, npart, jdone, {djd[0], djd[1]}, x32, N, vlen, R, nblk, nb,
                hstride, m};
    return hipMemcpyAsync(gsd, &gsh, sizeof(GsDev), hipMemcpyHostToDevice, s);
  }
  dim3 vgrid() const { return dim3((unsigned)nb, R); }
  unsigned lgrid(size_t len) const { return (unsigned)std::min<size_t>((len + 255) / 256, 4096); }
  // dots of the first J basis vectors with vec -> h (mode 0: h = dots; mode 3: h2 = dots, h += dots);
  // with flag, only for the RHS whose flag is set
  void mdot(const double2* Vb, int J, const double2* vec, double2* h, int mode, double2* h2 = nullptr,
            const int* flag = nullptr) {
    dim3 grid(nblk, (J + kDotVec - 1) / kDotVec, R);
    hipLaunchKernelGGL(mdot_kernel, grid, dim3(kDotThreads), 0, s, Vb, vlen, vec, N, J, part, flag);
    hipLaunchKernelGGL(mdot_finish, dim3((R * J + 3) / 4), dim3(256), 0, s, part, nblk, R, J, h, hstride, mode, h2,
                       flag);
  }
  // per-RHS 2-norm of vec into out[r][0]
  void norm(const double2* vec, double2* out) {
    hipLaunchKernelGGL(mdot_kernel, dim3(nblk, 1, R), dim3(kDotThreads), 0, s, vec, vlen, vec, N, 1, part,
                       (const int*)nullptr);
    hipLaunchKernelGGL(mdot_finish, dim3((R + 3) / 4), dim3(256), 0, s, part, nblk, R, 1, out, hstride, 2,
                       (double2*)nullptr, (const int*)nullptr);
  }
  // vec += sgn V c; with_norm: per-block |vec|^2 partials into npart; with flag, only flagged RHS
  void maxpy(const double2* Vb, const double2* c, double2* vec, int J, double sgn, bool with_norm = false,
             const int* flag = nullptr) {
    hipLaunchKernelGGL(maxpy_kernel, vgrid(), dim3(256), std::max(J, 1) * sizeof(double2), s, Vb, vlen, c, hstride,
                       vec, N, J, sgn, with_norm ? npart : nullptr, flag);
  }

  // back to the state before start() (a persistent solver runs several solves)
  void reset() {
    phase = RUN_TRUE;
    after_close = RUN_TRUE;
    j = 0;
    ++epoch;
    rec[0] = rec[1] = Rec{};
    its = refs = 0;
    ok = bad_input = false;
    emit = true;
    err = hipSuccess;
  }
  // ||b|| and ||x|| per RHS into the round slot's mapped norms (read by started() once that round
  // completed)
  void start(int slot) {
    norm(b, hn);
    hipLaunchKernelGGL(norm_out_kernel, dim3((R + 63) / 64), dim3(64), 0, s, hn, hstride, R, dres[slot]);
    norm(x, hn);
    hipLaunchKernelGGL(norm_out_kernel, dim3((R + 63) / 64), dim3(64), 0, s, hn, hstride, R, dres[slot] + R);
    rec[slot] = Rec{K_INIT, 0, epoch};
    phase = WAIT;
  }
  hipError_t started(int slot) {
    x_zero = true;
    for (int q = 0; q < R; ++q) {
      bn[q] = hres[slot][q];
      if (!std::isfinite(bn[q])) return hipErrorInvalidValue;
      if (hres[slot][R + q] != 0.0) x_zero = false;
    }
    if (ip == FMBEM_FP64) {
      gm_prec = FMBEM_FP64;
      gm_rhs = b;
      gm_sol = x;
      for (int q = 0; q < R; ++q) htol[q] = tol * bn[q];
      hipError_t e = hipMemcpyAsync(tolv, htol, R * sizeof(double), hipMemcpyHostToDevice, s);
      if (e) return e;
    } else {
      gm_prec = FMBEM_FP32;
      gm_rhs = rin;
      gm_sol = d;
    }
    phase = RUN_TRUE;
    return hipSuccess;
  }
  // end of a GMRES cycle: sol += V y with y = H^-1 g over each RHS's own step count
  void close_cycle() {
    hipLaunchKernelGGL(backsolve_kernel, dim3(R), dim3(256), (m + 1) * sizeof(double2), s, m, j, H, g, jdone, y,
                       hstride);
    maxpy(V, y, gm_sol, j, 1.0);
    ++epoch;
  }
  // cycle start on r (norm in hn): g, freeze flags, v_0 = r / beta (and its FP32 copy)
  void init_cycle(int slot) {
    hipLaunchKernelGGL(gmres_init_kernel, dim3((R + 63) / 64), dim3(64), 0, s, R, m, hn, hstride, tolv, g, jdone,
                       djd[slot], res);
    hipLaunchKernelGGL(scale_kernel, vgrid(), dim3(256), 0, s, r, hn, hstride, V,
                       gm_prec == FMBEM_FP32 ? x32 : nullptr, N);
    j = 0;
  }

  void pre(int slot) {
    req = false;
    rec[slot] = Rec{};
    if (phase == DONE || phase == WAIT) return;
    if (phase == CLOSE) {
      close_cycle();
      if (after_close == RUN_TRUE && ip == FMBEM_FP32)
        hipLaunchKernelGGL(add_kernel, dim3(lgrid(vlen)), dim3(256), 0, s, x, d, vlen);
      phase = after_close;
    }
    if (phase == START_INNER) {
      // inner system A32 d = r from d = 0: the residual norm of the true-residual step is beta
      hipLaunchKernelGGL(zero_kernel, dim3(lgrid(vlen)), dim3(256), 0, s, d, vlen);
      hipLaunchKernelGGL(copy_kernel, dim3(lgrid(vlen)), dim3(256), 0, s, rin, r, vlen);
      init_cycle(slot);
      phase = RUN_ARN;
    }
    switch (phase) {
      case RUN_TRUE:
        if (x_zero) {
          // zero initial guess: A x = 0, the first true residual is b without an operator application
          hipLaunchKernelGGL(zero_kernel, dim3(lgrid(vlen)), dim3(256), 0, s, t, vlen);
          x_zero = false;
        } else {
          req = true;
          req_prec = FMBEM_FP64;
          req_in = x;
          req_out = t;
        }
        rec[slot] = Rec{K_TRUE, 0, epoch};
        break;
      case RUN_RESTART:
        hipLaunchKernelGGL(to32_kernel, dim3(lgrid(vlen)), dim3(256), 0, s, d, x32, vlen);
        req = true;
        req_prec = FMBEM_FP32;
        req_in = x32;
        req_out = t;
        rec[slot] = Rec{K_RESTART, 0, epoch};
        break;
      case RUN_ARN:
        // the FP32 copy of v_j was written by the kernel that produced v_j
        req = true;
        req_prec = gm_prec;
        req_in = gm_prec == FMBEM_FP32 ? (const void*)x32 : (const void*)(V + (size_t)j * vlen);
        req_out = V + (size_t)(j + 1) * vlen;  // w = A v_j is built in the slot of v_{j+1}
        rec[slot] = Rec{K_ARN, j, epoch};
        break;
      default:
        break;
    }
  }

  // grouped: this step's single-pass Gram-Schmidt is launched by the caller together with other
  // members' (gs_group_launch)
  bool gs_groupable(int slot) const { return rec[slot].kind == K_ARN && emit && ortho == FMBEM_ORTHO_ONCE; }
  void post(int slot, bool grouped = false) {
    switch (rec[slot].kind) {
      case K_TRUE:
        hipLaunchKernelGGL(sub_kernel, dim3(lgrid(vlen)), dim3(256), 0, s, b, t, r, vlen);
        norm(r, hn);
        hipLaunchKernelGGL(norm_out_kernel, dim3((R + 63) / 64), dim3(64), 0, s, hn, hstride, R, dres[slot]);
        if (ip == FMBEM_FP64) init_cycle(slot);  // the true residual starts the next cycle
        phase = WAIT;
        break;
      case K_RESTART:
        hipLaunchKernelGGL(sub_kernel, dim3(lgrid(vlen)), dim3(256), 0, s, rin, t, r, vlen);
        norm(r, hn);
        init_cycle(slot);
        phase = RUN_ARN;
        break;
      case K_ARN: {
        if (emit && !grouped) {
          double2* wv = V + (size_t)(j + 1) * vlen;
          // Gram-Schmidt: h = V^H w (and ||w||^2 as the last dot), w -= V h (with |w|^2 partials);
          // second pass h2 = V^H w, w -= V h2, h += h2 where the DGKS criterion (or the mode) asks for it
          mdot(V, j + 2, wv, hc, 0);
          maxpy(V, hc, wv, j + 1, -1.0, true);
          if (ortho != FMBEM_ORTHO_ONCE) {
            hipLaunchKernelGGL(reorth_check_kernel, dim3(R), dim3(256), 0, s, ortho, nb, npart, hc, hstride, j, jdone,
                               reorth);
            mdot(V, j + 1, wv, hc, 3, y, reorth);
            maxpy(V, y, wv, j + 1, -1.0, true, reorth);
          }
          hipLaunchKernelGGL(scale_givens_kernel, vgrid(), dim3(256), (3 * m + 2) * sizeof(double2), s, npart, nb, m,
                             j, hc, hstride, hn, H, cs,
                             sn, g, res, jdone, djd[slot], tolv, wv, gm_prec == FMBEM_FP32 ? x32 : nullptr, N);
        }
        ++its;
        ++j;
        // a full cycle (or the iteration budget) ends here; what follows needs this step's flags
        if (j == m || its >= max_its) phase = WAIT;
        break;
      }
      default:
        break;
    }
  }

  // host: results of the step queued in round slot (its event has completed)
  void process(int slot) {
    const Rec rc = rec[slot];
    if (rc.kind == K_NONE || phase == DONE || rc.epoch != epoch) return;
    if (rc.kind == K_INIT) {
      const hipError_t e = started(slot);
      if (e == hipErrorInvalidValue) {
        bad_input = true;  // non-finite ||b||: this problem ends, the others go on
        phase = DONE;
      } else {
        err = e;
      }
      return;
    }
    if (rc.kind == K_TRUE) {
      ok = true;
      for (int q = 0; q < R; ++q) {
        rel[q] = bn[q] > 0 ? hres[slot][q] / bn[q] : 0.0;
        if (!(rel[q] <= tol)) ok = false;
      }
      if (ok || its >= max_its || (ip == FMBEM_FP32 && refs >= max_ref)) {
        phase = DONE;
        return;
      }
      if (ip == FMBEM_FP64) {
        phase = RUN_ARN;  // the cycle was started by the true-residual step
      } else {
        // inner tolerance: inner_tol * ||r||, and not below what the outer test needs
        for (int q = 0; q < R; ++q) htol[q] = std::max(inner_tol * rel[q] * bn[q], 0.5 * tol * bn[q]);
        hipError_t e = hipMemcpyAsync(tolv, htol, R * sizeof(double), hipMemcpyHostToDevice, s);
        if (e) err = e;
        ++refs;
        phase = START_INNER;
      }
      return;
    }
    // K_RESTART (flags of the cycle start) or K_ARN (flags after step rc.j)
    bool all = true;
    for (int q = 0; q < R; ++q)
      if (hjd[slot][q] < 0) all = false;
    const bool last = rc.kind == K_ARN && (rc.j + 1 == m || its >= max_its) && rc.j + 1 == j;
    if (all || last) {
      // close the cycle; in FP32 mode the inner solve ends when it converged or the budget is spent
      phase = CLOSE;
      after_close = (ip == FMBEM_FP64 || all || its >= max_its) ? RUN_TRUE : RUN_RESTART;
      if (rc.kind == K_ARN && !all) j = rc.j + 1;  // steps of this cycle (all of them were processed)
    }
  }
};

static fmbem_status st_of(hipError_t e) {
  if (e == hipSuccess) return FMBEM_OK;
  return e == hipErrorOutOfMemory ? FMBEM_ERR_OUT_OF_MEMORY : FMBEM_ERR_DEVICE;
}

// validated solve options (defaults filled in)
struct SolveCfg {
  double tol, inner_tol;
  int m, max_its, max_ref, ip, ortho;
};
static fmbem_status solve_cfg(const Plan& P, const fmbem_solve_opts* opts, int n_rhs, SolveCfg& c) {
  if (!opts || n_rhs < 1) return FMBEM_ERR_INVALID_ARG;
  if (!(opts->tol > 0.0) || !std::isfinite(opts->tol)) return FMBEM_ERR_INVALID_ARG;
  c.tol = opts->tol;
  c.m = opts->restart == 0 ? 30 : opts->restart;
  if (c.m < 1 || c.m > kMaxRestart) return FMBEM_ERR_INVALID_ARG;
  c.max_its = opts->max_iters == 0 ? 1000 : opts->max_iters;
  c.max_ref = opts->max_refinements == 0 ? 20 : opts->max_refinements;
  c.inner_tol = opts->inner_tol == 0.0 ? 1e-5 : opts->inner_tol;
  if (c.max_its < 1 || c.max_ref < 1 || !(c.inner_tol > 0.0) || c.inner_tol >= 1.0) return FMBEM_ERR_INVALID_ARG;
  c.ip = opts->inner_precision;
  if (c.ip != FMBEM_FP64 && c.ip != FMBEM_FP32) return FMBEM_ERR_INVALID_ARG;
  c.ortho = opts->orthogonalization;
  if (c.ortho < FMBEM_ORTHO_DGKS || c.ortho > FMBEM_ORTHO_ONCE) return FMBEM_ERR_INVALID_ARG;
  if (!(P.precisions & 1u)) return FMBEM_ERR_UNSUPPORTED;  // the true residual needs the FP64 operator
  if (c.ip == FMBEM_FP32 && !(P.precisions & 2u)) return FMBEM_ERR_UNSUPPORTED;
  if ((size_t)n_rhs * P.C > (size_t)INT32_MAX / 2) return FMBEM_ERR_UNSUPPORTED;
  return FMBEM_OK;
}

static void configure(Member& mb, const SolveCfg& c, const void* b, void* x) {
  mb.ortho = c.ortho;
  mb.ip = c.ip;
  mb.tol = c.tol;
  mb.inner_tol = c.inner_tol;
  mb.max_its = c.max_its;
  mb.max_ref = c.max_ref;
  mb.b = reinterpret_cast<const double2*>(b);
  mb.x = reinterpret_cast<double2*>(x);
}

// single-pass Gram-Schmidt steps of several members, each kernel once per kMaxGsJobs steps
struct GsStep {
  const GsDev* d;
  const GsDev* h;
  int j, mode;
};
static hipError_t gs_group_launch(const std::vector<GsStep>& v, hipStream_t s) {
  for (size_t i0 = 0; i0 < v.size(); i0 += kMaxGsJobs) {
    const size_t i1 = std::min(v.size(), i0 + kMaxGsJobs);
    for (int kernel = 0; kernel < 4; ++kernel) {
      GsJobs J{};
      int blocks = 0;
      size_t lds = 0;
      for (size_t i = i0; i < i1; ++i) {
        J.d[J.count] = v[i].d;
        J.j[J.count] = v[i].j;
        J.mode[J.count] = v[i].mode;
        J.block0[J.count++] = blocks;
        blocks += gs_blocks(kernel, *v[i].h, v[i].j);
        if (kernel == 2) lds = std::max(lds, (size_t)(v[i].j + 1) * sizeof(double2));
        if (kernel == 3) lds = std::max(lds, (size_t)(3 * v[i].h->m + 2) * sizeof(double2));
      }
      J.block0[J.count] = blocks;
      if (kernel == 0) hipLaunchKernelGGL(gs_mdot_kernel, dim3(blocks), dim3(kDotThreads), 0, s, J);
      else if (kernel == 1) hipLaunchKernelGGL(gs_finish_kernel, dim3(blocks), dim3(256), 0, s, J);
      else if (kernel == 2) hipLaunchKernelGGL(gs_maxpy_kernel, dim3(blocks), dim3(256), lds, s, J);
      else hipLaunchKernelGGL(gs_scale_givens_kernel, dim3(blocks), dim3(256), lds, s, J);
      const hipError_t e = hipGetLastError();
      if (e) return e;
    }
  }
  return hipSuccess;
}

// The work of one round: pre() of every member, the members' operator applications in
// grouped launches (one sequence per precision), post() of every member.
static hipError_t round_enqueue(const std::vector<Member*>& ms, int slot, hipStream_t s, bool tune) {
  std::vector<GroupApply> g64, g32;
  for (Member* mb : ms) {
    mb->pre(slot);
    if (!mb->req) continue;
    const bool f32 = mb->req_prec == FMBEM_FP32;
    GroupApply a{&mb->P, mb->R, mb->req_in, f32 ? nullptr : (void*)mb->req_out, mb->ws,
                 f32 ? (void*)mb->req_out : nullptr};
    (f32 ? g32 : g64).push_back(a);
  }
  hipError_t e = matvec_group(FMBEM_FP64, g64, s, tune);
  if (!e) e = matvec_group(FMBEM_FP32, g32, s, tune);
  if (e) return e;
  std::vector<GsStep> gs;
  for (Member* mb : ms)
    if (mb->gs_groupable(slot))
      gs.push_back(GsStep{mb->gsd, &mb->gsh, mb->j, slot | (mb->gm_prec == FMBEM_FP32 ? 2 : 0)});
  const bool grouped = gs.size() >= 2;
  for (Member* mb : ms) mb->post(slot, grouped && mb->gs_groupable(slot));
  if (grouped && (e = gs_group_launch(gs, s))) return e;
  return hipGetLastError();
}

// End of round t: its event, then the host reads round t-1's results (which finished
// while round t runs).
static hipError_t round_finish(const std::vector<Member*>& ms, long long t, hipStream_t s, hipEvent_t ev[2]) {
  const int slot = (int)(t & 1);
  hipError_t e;
  if ((e = hipEventRecord(ev[slot], s))) return e;
  if (t > 0) {
    if ((e = hipEventSynchronize(ev[slot ^ 1]))) return e;
    for (Member* mb : ms) {
      mb->process(slot ^ 1);
      if (mb->err) return mb->err;
    }
  }
  return hipSuccess;
}

// Solve every member to completion in lockstep rounds.
static hipError_t run_group(const std::vector<Member*>& ms, hipStream_t s, bool tune) {
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2 && !e; ++i) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
  if (!e) {
    for (Member* mb : ms) mb->start(0);
    e = hipStreamSynchronize(s);
    for (Member* mb : ms) {
      if (!e) e = mb->started(0);
      mb->rec[0] = Member::Rec{};
    }
  }
  for (long long t = 0; !e; ++t) {
    bool live = false;
    for (Member* mb : ms)
      if (mb->phase != Member::DONE) live = true;
    if (!live) break;
    e = round_enqueue(ms, (int)(t & 1), s, tune);
    if (!e) e = round_finish(ms, t, s, ev);
  }
  if (!e) e = hipStreamSynchronize(s);
  for (int i = 0; i < 2; ++i)
    if (ev[i]) hipEventDestroy(ev[i]);
  return e;
}

static void fill_info(const Member& mb, fmbem_solve_info* info) {
  for (int q = 0; q < mb.R; ++q) {
    info[q].iterations = mb.its;
    info[q].refinements = mb.refs;
    info[q].rel_residual = mb.rel[q];
  }
}

// Serving engine: continuous batching of solve requests.  Requests queue in arrival
// order; at the start of every step the queue head is admitted while a slot is free
// and its device footprint (Krylov basis, work vectors, operator workspace) fits the
// byte budget.  A step is one round (see Member) over every admitted problem, whose
// operator applications share grouped launches; finished problems free their memory
// and leave their results for poll().  Plans stay resident with their owners.
struct Engine {
  hipStream_t s = nullptr;
  size_t budget = 0;
  int max_slots = 1;
  size_t used = 0;
  long long next_ticket = 1;
  long long t = 0;  // rounds
  struct Req {
    long long ticket;
    const Plan* P;
    SolveCfg c;
    int R;
    const void* b;
    void* x;
    size_t bytes;
  };
  std::deque<Req> queue;
  struct Slot {
    std::unique_ptr<Member> mb;
    long long ticket;
    size_t bytes;
  };
  std::vector<Slot> active;
  struct Result {
    fmbem_status st;
    std::vector<fmbem_solve_info> info;
  };
  std::unordered_map<long long, Result> results;
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::mutex mu;
  fmbem_engine_timing timing{};
  // device memory of the problems: stream-ordered allocations from the engine's own pool, which
  // keeps freed memory for the next problem (no device-wide synchronisation at admission or
  // retirement); nullptr where pools are unavailable (plain allocations then)
  hipMemPool_t pool = nullptr;
  // plans of the active problems (a plan's resident bytes count once against the budget while
  // any of its problems is active)
  std::unordered_map<const Plan*, int> plan_refs;

  ~Engine() {
    hipStreamSynchronize(s);
    active.clear();
    hipStreamSynchronize(s);
    for (int i = 0; i < 2; ++i)
      if (ev[i]) hipEventDestroy(ev[i]);
    if (pool) hipMemPoolDestroy(pool);
  }

  hipError_t make_pool() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e) return e;
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    if (hipMemPoolCreate(&pool, &props) != hipSuccess) {
      (void)hipGetLastError();
      pool = nullptr;  // plain allocations
      return hipSuccess;
    }
    uint64_t keep = UINT64_MAX;
    return hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }

  // bytes a request adds to the budget when admitted: its buffers, and its plan unless counted
  size_t admit_bytes(const Req& q) const {
    auto it = plan_refs.find(q.P);
    return q.bytes + ((it == plan_refs.end() || it->second == 0) ? q.P->resident : 0);
  }

  static size_t footprint(const Plan& P, const SolveCfg& c, int R) {
    Member probe(P, nullptr, R, c.m);
    return probe.footprint(c.ip == FMBEM_FP32);
  }

  void finish(Slot& sl, fmbem_status st) {
    Result r{st, std::vector<fmbem_solve_info>(sl.mb->R)};
    fill_info(*sl.mb, r.info.data());
    results[sl.ticket] = std::move(r);
    used -= sl.bytes;
    const Plan* P = &sl.mb->P;
    if (--plan_refs[P] == 0) {
      used -= P->resident;
      plan_refs.erase(P);
    }
    sl.mb.reset();
  }

  static double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
  }
  hipError_t step() {
    std::vector<Member*> ms;
    for (Slot& sl : active) ms.push_back(sl.mb.get());
    const int slot = (int)(t & 1);
    double t0 = now();
    hipError_t e = round_enqueue(ms, slot, s, false);
    if (e) return e;
    double t1 = now();
    timing.enqueue_s += t1 - t0;
    if (!ms.empty()) {
      ++timing.rounds;
      timing.member_rounds += (int64_t)ms.size();
    }
    // admission in arrival order: the queue head waits until it fits
    while (!queue.empty() && (int)active.size() < max_slots && used + admit_bytes(queue.front()) <= budget) {
      Req q = queue.front();
      queue.pop_front();
      Slot sl{std::unique_ptr<Member>(new Member(*q.P, s, q.R, q.c.m)), q.ticket, q.bytes};
      configure(*sl.mb, q.c, q.b, q.x);
      e = sl.mb->setup(q.c.ip == FMBEM_FP32, pool);
      if (e) {
        results[q.ticket] = Result{st_of(e), std::vector<fmbem_solve_info>(q.R)};
        if (e == hipErrorOutOfMemory) {
          (void)hipGetLastError();
          continue;
        }
        return e;
      }
      sl.mb->start(slot);
      used += q.bytes;
      if (plan_refs[q.P]++ == 0) used += q.P->resident;
      ms.push_back(sl.mb.get());
      active.push_back(std::move(sl));
      ++timing.admitted;
    }
    double t2 = now();
    timing.admit_s += t2 - t1;
    if ((e = round_finish(ms, t, s, ev))) return e;
    ++t;
    double t3 = now();
    timing.wait_s += t3 - t2;
    // retire: a finished problem has no work in flight (its last step was the true residual
    // read above, and it queued nothing since)
    for (Slot& sl : active)
      if (sl.mb->phase == Member::DONE) {
        finish(sl, sl.mb->bad_input ? FMBEM_ERR_INVALID_ARG : (sl.mb->ok ? FMBEM_OK : FMBEM_ERR_NOT_CONVERGED));
        ++timing.retired;
      }
    active.erase(std::remove_if(active.begin(), active.end(), [](const Slot& sl) { return !sl.mb; }), active.end());
    timing.retire_s += now() - t3;
    return hipSuccess;
  }
};

// Persistent solver: one Member whose buffers live across solves, on an internal stream
// (ordered after the caller's stream on entry; the call blocks until done).  With graphs,
// every pure Arnoldi round (no cycle start or end in it) is captured once per (Arnoldi index,
// round parity) after it ran eagerly once (so that tile shapes are tuned), and later rounds
// with the same key replay the graph while the host state advances as in an eager round.
// b and x are staged in the solver's own buffers so that the graphs see fixed addresses.
struct Solver {
  const Plan& P;
  SolveCfg c;
  int R;
  bool graphs = false;
  hipStream_t si = nullptr;
  std::unique_ptr<Member> mb;
  double2* bbuf = nullptr;
  double2* xbuf = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t join = nullptr;
  std::map<std::pair<int, int>, int> seen;
  std::map<std::pair<int, int>, hipGraphExec_t> execs;
  long long replays = 0;

  Solver(const Plan& p, const SolveCfg& c_, int R_) : P(p), c(c_), R(R_) {}
  ~Solver() {
    if (si) hipStreamSynchronize(si);
    for (auto& kv : execs) hipGraphExecDestroy(kv.second);
    mb.reset();
    if (bbuf) hipFree(bbuf);
    if (xbuf) hipFree(xbuf);
    for (int i = 0; i < 2; ++i)
      if (ev[i]) hipEventDestroy(ev[i]);
    if (join) hipEventDestroy(join);
    if (si) hipStreamDestroy(si);
  }
  hipError_t setup() {
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&si, hipStreamNonBlocking))) return e;
    for (int i = 0; i < 2; ++i)
      if ((e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming))) return e;
    if ((e = hipEventCreateWithFlags(&join, hipEventDisableTiming))) return e;
    mb.reset(new Member(P, si, R, c.m));
    const size_t vb = (size_t)R * P.n * P.C * sizeof(double2);
    if ((e = hipMalloc((void**)&bbuf, vb))) return e;
    if ((e = hipMalloc((void**)&xbuf, vb))) return e;
    configure(*mb, c, bbuf, xbuf);
    return mb->setup(c.ip == FMBEM_FP32);
  }
  // one round, eager, captured, or replayed
  hipError_t round(long long t) {
    Member& m = *mb;
    const int slot = (int)(t & 1);
    const bool pure = graphs && m.phase == Member::RUN_ARN && P.prof.mask == 0;
    if (!pure) return round_enqueue({&m}, slot, si, true);
    const std::pair<int, int> key{m.j, slot};
    auto it = execs.find(key);
    if (it != execs.end()) {
      m.emit = false;
      m.pre(slot);
      m.post(slot);
      m.emit = true;
      ++replays;
      return hipGraphLaunch(it->second, si);
    }
    if (seen[key]++ == 0) return round_enqueue({&m}, slot, si, true);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamBeginCapture(si, hipStreamCaptureModeThreadLocal);
    if (e) return e;
    const hipError_t er = round_enqueue({&m}, slot, si, true);
    e = hipStreamEndCapture(si, &gr);
    if (er) {
      if (gr) hipGraphDestroy(gr);
      return er;
    }
    if (e) return e;
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    hipGraphDestroy(gr);
    if (e) return e;
    execs[key] = ex;
    return hipGraphLaunch(ex, si);
  }
  hipError_t run(const void* b, void* x, hipStream_t caller) {
    const size_t vb = (size_t)R * P.n * P.C * sizeof(double2);
    hipError_t e;
    if ((e = hipEventRecord(join, caller))) return e;
    if ((e = hipStreamWaitEvent(si, join, 0))) return e;
    if ((e = hipMemcpyAsync(bbuf, b, vb, hipMemcpyDeviceToDevice, si))) return e;
    if ((e = hipMemcpyAsync(xbuf, x, vb, hipMemcpyDeviceToDevice, si))) return e;
    Member& m = *mb;
    m.reset();
    m.start(0);
    if ((e = hipStreamSynchronize(si))) return e;
    if ((e = m.started(0))) return e;
    m.rec[0] = Member::Rec{};
    for (long long t = 0; m.phase != Member::DONE; ++t) {
      if ((e = round(t))) return e;
      if ((e = round_finish({&m}, t, si, ev))) return e;
    }
    if ((e = hipMemcpyAsync(x, xbuf, vb, hipMemcpyDeviceToDevice, si))) return e;
    return hipStreamSynchronize(si);
  }
};

}  // namespace fmbem

using namespace fmbem;

extern "C" fmbem_status fmbem_solve(fmbem_plan plan, const fmbem_solve_opts* opts, int32_t n_rhs, const void* b,
                                    void* x, fmbem_solve_info* info, void* hip_stream) {
  if (!plan || !opts || !b || !x || n_rhs < 1) return FMBEM_ERR_INVALID_ARG;
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  SolveCfg c;
  fmbem_status st = solve_cfg(P, opts, n_rhs, c);
  if (st != FMBEM_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  Member mb(P, s, n_rhs, c.m);
  configure(mb, c, b, x);
  hipError_t e = mb.setup(c.ip == FMBEM_FP32);
  if (e) return st_of(e);
  e = run_group({&mb}, s, true);
  if (e == hipErrorInvalidValue) return FMBEM_ERR_INVALID_ARG;  // non-finite b
  if (e) return st_of(e);
  if (info) fill_info(mb, info);
  return mb.ok ? FMBEM_OK : FMBEM_ERR_NOT_CONVERGED;
}

extern "C" fmbem_status fmbem_solve_batch(int32_t n, const fmbem_plan* plans, const fmbem_solve_opts* opts,
                                          const int32_t* n_rhs, const void* const* b, void* const* x,
                                          fmbem_solve_info* info, void* hip_stream) {
  if (n < 1 || !plans || !opts || !n_rhs || !b || !x) return FMBEM_ERR_INVALID_ARG;
  std::vector<SolveCfg> cfg(n);
  for (int i = 0; i < n; ++i) {
    if (!plans[i] || !b[i] || !x[i]) return FMBEM_ERR_INVALID_ARG;
    fmbem_status st = solve_cfg(*reinterpret_cast<Plan*>(plans[i]), &opts[i], n_rhs[i], cfg[i]);
    if (st != FMBEM_OK) return st;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  std::vector<std::unique_ptr<Member>> own;
  std::vector<Member*> ms;
  for (int i = 0; i < n; ++i) {
    own.emplace_back(new Member(*reinterpret_cast<Plan*>(plans[i]), s, n_rhs[i], cfg[i].m));
    configure(*own.back(), cfg[i], b[i], x[i]);
    hipError_t e = own.back()->setup(cfg[i].ip == FMBEM_FP32);
    if (e) return st_of(e);
    ms.push_back(own.back().get());
  }
  hipError_t e = run_group(ms, s, true);
  if (e == hipErrorInvalidValue) return FMBEM_ERR_INVALID_ARG;
  if (e) return st_of(e);
  bool ok = true;
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    if (info) fill_info(*ms[i], info + off);
    off += n_rhs[i];
    if (!ms[i]->ok) ok = false;
  }
  return ok ? FMBEM_OK : FMBEM_ERR_NOT_CONVERGED;
}

extern "C" fmbem_status fmbem_engine_create(size_t hbm_budget_bytes, int32_t max_slots, void* hip_stream,
                                            fmbem_engine* out) {
  if (!out || max_slots < 1 || hbm_budget_bytes == 0) return FMBEM_ERR_INVALID_ARG;
  *out = nullptr;
  std::unique_ptr<Engine> e(new Engine);
  e->s = reinterpret_cast<hipStream_t>(hip_stream);
  e->budget = hbm_budget_bytes;
  e->max_slots = max_slots;
  for (int i = 0; i < 2; ++i)
    if (hipEventCreateWithFlags(&e->ev[i], hipEventDisableTiming) != hipSuccess) return FMBEM_ERR_DEVICE;
  if (e->make_pool() != hipSuccess) return FMBEM_ERR_DEVICE;
  *out = reinterpret_cast<fmbem_engine>(e.release());
  return FMBEM_OK;
}

extern "C" fmbem_status fmbem_engine_submit(fmbem_engine engine, fmbem_plan plan, const fmbem_solve_opts* opts,
                                            int32_t n_rhs, const void* b, void* x, int64_t* ticket) {
  if (!engine || !plan || !opts || !b || !x || !ticket || n_rhs < 1) return FMBEM_ERR_INVALID_ARG;
  Engine& E = *reinterpret_cast<Engine*>(engine);
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  SolveCfg c;
  const fmbem_status st = solve_cfg(P, opts, n_rhs, c);
  if (st != FMBEM_OK) return st;
  const size_t bytes = Engine::footprint(P, c, n_rhs);
  std::lock_guard<std::mutex> lk(E.mu);
  if (bytes + P.resident > E.budget) return FMBEM_ERR_ADMISSION;
  *ticket = E.next_ticket++;
  E.queue.push_back(Engine::Req{*ticket, &P, c, n_rhs, b, x, bytes});
  return FMBEM_OK;
}

extern "C" fmbem_status fmbem_engine_step(fmbem_engine engine) {
  if (!engine) return FMBEM_ERR_INVALID_ARG;
  Engine& E = *reinterpret_cast<Engine*>(engine);
  std::lock_guard<std::mutex> lk(E.mu);
  if (E.active.empty() && E.queue.empty()) return FMBEM_OK;
  return st_of(E.step());
}

extern "C" fmbem_status fmbem_engine_poll(fmbem_engine engine, int64_t ticket, int32_t* done,
                                          fmbem_solve_info* info) {
  if (!engine || !done) return FMBEM_ERR_INVALID_ARG;
  Engine& E = *reinterpret_cast<Engine*>(engine);
  std::lock_guard<std::mutex> lk(E.mu);
  auto it = E.results.find(ticket);
  if (it == E.results.end()) {
    if (ticket < 1 || ticket >= E.next_ticket) return FMBEM_ERR_INVALID_ARG;
    bool known = false;
    for (const auto& q : E.queue)
      if (q.ticket == ticket) known = true;
    for (const auto& sl : E.active)
      if (sl.ticket == ticket) known = true;
    if (!known) return FMBEM_ERR_INVALID_ARG;  // already collected
    *done = 0;
    return FMBEM_OK;
  }
  *done = 1;
  if (info) std::copy(it->second.info.begin(), it->second.info.end(), info);
  const fmbem_status st = it->second.st;
  E.results.erase(it);
  return st;
}

extern "C" fmbem_status fmbem_engine_stats(fmbem_engine engine, int32_t* active, int32_t* queued,
                                           size_t* bytes_in_use) {
  if (!engine) return FMBEM_ERR_INVALID_ARG;
  Engine& E = *reinterpret_cast<Engine*>(engine);
  std::lock_guard<std::mutex> lk(E.mu);
  if (active) *active = (int32_t)E.active.size();
  if (queued) *queued = (int32_t)E.queue.size();
  if (bytes_in_use) *bytes_in_use = E.used;
  return FMBEM_OK;
}

extern "C" fmbem_status fmbem_engine_timing_read(fmbem_engine engine, fmbem_engine_timing* out) {
  if (!engine || !out) return FMBEM_ERR_INVALID_ARG;
  Engine& E = *reinterpret_cast<Engine*>(engine);
  std::lock_guard<std::mutex> lk(E.mu);
  *out = E.timing;
  return FMBEM_OK;
}

extern "C" fmbem_status fmbem_engine_destroy(fmbem_engine engine) {
  if (!engine) return FMBEM_ERR_INVALID_ARG;
  delete reinterpret_cast<Engine*>(engine);
  return FMBEM_OK;
}

extern "C" fmbem_status fmbem_solver_create(fmbem_plan plan, const fmbem_solve_opts* opts, int32_t n_rhs,
                                            int32_t use_graphs, fmbem_solver* out) {
  if (!plan || !opts || !out || n_rhs < 1 || (use_graphs != 0 && use_graphs != 1)) return FMBEM_ERR_INVALID_ARG;
  *out = nullptr;
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  SolveCfg c;
  const fmbem_status st = solve_cfg(P, opts, n_rhs, c);
  if (st != FMBEM_OK) return st;
  std::unique_ptr<Solver> sv(new Solver(P, c, n_rhs));
  sv->graphs = use_graphs == 1;
  const hipError_t e = sv->setup();
  if (e) return st_of(e);
  *out = reinterpret_cast<fmbem_solver>(sv.release());
  return FMBEM_OK;
}

extern "C" fmbem_status fmbem_solver_run(fmbem_solver solver, const void* b, void* x, fmbem_solve_info* info,
                                         void* hip_stream) {
  if (!solver || !b || !x) return FMBEM_ERR_INVALID_ARG;
  Solver& sv = *reinterpret_cast<Solver*>(solver);
  const hipError_t e = sv.run(b, x, reinterpret_cast<hipStream_t>(hip_stream));
  if (e == hipErrorInvalidValue) return FMBEM_ERR_INVALID_ARG;
  if (e) return st_of(e);
  if (info) fill_info(*sv.mb, info);
  return sv.mb->ok ? FMBEM_OK : FMBEM_ERR_NOT_CONVERGED;
}

extern "C" fmbem_status fmbem_solver_graph_stats(fmbem_solver solver, int32_t* graphs, int64_t* replays) {
  if (!solver) return FMBEM_ERR_INVALID_ARG;
  const Solver& sv = *reinterpret_cast<Solver*>(solver);
  if (graphs) *graphs = (int32_t)sv.execs.size();
  if (replays) *replays = sv.replays;
  return FMBEM_OK;
}

extern "C" fmbem_status fmbem_solver_destroy(fmbem_solver solver) {
  if (!solver) return FMBEM_ERR_INVALID_ARG;
  delete reinterpret_cast<Solver*>(solver);
  return FMBEM_OK;
}
