// Restarted GMRES with FP64 Arnoldi (classical Gram-Schmidt applied twice),
// Givens rotations and FP64 iterative refinement around FP32 inner solves.
//
// The paper solves the FMPBEM system iteratively with GMRES (Sec. 2.4, Sec. 3.5,
// Sec. 4).  All right-hand sides are iterated together, each in its own Krylov
// space; vectors are [R][N] complex128.  Per Arnoldi step:
//   w = A v_j                         (operator in FP64, or FP32 through casts)
//   h = V^H w, w -= V h  (twice)      (multi-dot and multi-axpy kernels, FP64)
//   h_{j+1} = ||w||, v_{j+1} = w / h_{j+1}
//   Givens update of the Hessenberg column and of g on the device (one thread per RHS)
// Only the per-RHS residual estimates |g_{j+1}| cross to the host each step.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace fmbem {

constexpr int kEl = 4;          // elements per thread in the multi-dot kernel
constexpr int kDotThreads = 256;

__device__ inline double2 warp_sum(double2 v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_down(v.x, o, 64);
    v.y += __shfl_down(v.y, o, 64);
  }
  return v;
}

// part[r][i][blk] = sum_{n in block} conj(V_i[r][n]) w[r][n], i < J
__global__ __launch_bounds__(kDotThreads) void mdot_kernel(const double2* __restrict__ V, size_t vstride,
                                                           const double2* __restrict__ w, size_t N, int R, int J,
                                                           double2* __restrict__ part) {
  __shared__ double2 red[kDotThreads / 64];
  const int r = blockIdx.y;
  const int nblk = gridDim.x;
  const size_t base = (size_t)blockIdx.x * kDotThreads * kEl;
  double2 wl[kEl];
#pragma unroll
  for (int e = 0; e < kEl; ++e) {
    const size_t n = base + e * kDotThreads + threadIdx.x;
    wl[e] = n < N ? w[(size_t)r * N + n] : make_double2(0, 0);
  }
  for (int i = 0; i < J; ++i) {
    const double2* vi = V + i * vstride + (size_t)r * N;
    double2 acc = make_double2(0, 0);
#pragma unroll
    for (int e = 0; e < kEl; ++e) {
      const size_t n = base + e * kDotThreads + threadIdx.x;
      if (n < N) {
        const double2 a = vi[n];
        acc.x += a.x * wl[e].x + a.y * wl[e].y;
        acc.y += a.x * wl[e].y - a.y * wl[e].x;
      }
    }
    acc = warp_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double2 s = red[0];
      for (int t = 1; t < kDotThreads / 64; ++t) { s.x += red[t].x; s.y += red[t].y; }
      part[((size_t)r * J + i) * nblk + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// h[r][i] (+)= sum_blk part[r][i][blk]; mode 0: set, 1: add, 2: store norm sqrt(re) into h[r][i]
__global__ void mdot_finish(const double2* __restrict__ part, int nblk, int R, int J, double2* __restrict__ h,
                            int hstride, int mode) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= R * J) return;
  const int r = t / J, i = t - r * J;
  double2 s = make_double2(0, 0);
  for (int b = 0; b < nblk; ++b) {
    const double2 v = part[(size_t)t * nblk + b];
    s.x += v.x;
    s.y += v.y;
  }
  double2* o = h + (size_t)r * hstride + i;
  if (mode == 0) *o = s;
  else if (mode == 1) { o->x += s.x; o->y += s.y; }
  else *o = make_double2(sqrt(fmax(s.x, 0.0)), 0.0);
}

// w[r][n] += sgn * sum_{i<J} c[r][i] V_i[r][n]
__global__ void maxpy_kernel(const double2* __restrict__ V, size_t vstride, const double2* __restrict__ c,
                             int cstride, double2* __restrict__ w, size_t N, int R, int J, double sgn) {
  extern __shared__ double2 cs[];
  const int r = blockIdx.y;
  for (int i = threadIdx.x; i < J; i += blockDim.x) cs[i] = c[(size_t)r * cstride + i];
  __syncthreads();
  for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (size_t)gridDim.x * blockDim.x) {
    double2 acc = w[(size_t)r * N + n];
    for (int i = 0; i < J; ++i) {
      const double2 v = V[i * vstride + (size_t)r * N + n];
      acc.x += sgn * (cs[i].x * v.x - cs[i].y * v.y);
      acc.y += sgn * (cs[i].x * v.y + cs[i].y * v.x);
    }
    w[(size_t)r * N + n] = acc;
  }
}

// out[r][n] = a[r][n] * s[r]  (s real, from the .x of a double2 array)
__global__ void scale_kernel(const double2* __restrict__ a, const double2* __restrict__ s, int sstride,
                             double2* __restrict__ out, size_t N, int R, int invert) {
  const int r = blockIdx.y;
  double f = s[(size_t)r * sstride].x;
  f = invert ? (f > 0 ? 1.0 / f : 0.0) : f;
  for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (size_t)gridDim.x * blockDim.x) {
    const double2 v = a[(size_t)r * N + n];
    out[(size_t)r * N + n] = make_double2(v.x * f, v.y * f);
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

__global__ void to32_kernel(const double2* __restrict__ a, float2* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

__global__ void to64_kernel(const float2* __restrict__ a, double2* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = make_double2((double)a[i].x, (double)a[i].y);
}

// Hessenberg column j from hc (j+1 coefficients) and the norm hn; Givens rotations
// [[conj(c), conj(s)], [-s, c]]; g update; residual estimate.  One thread per RHS.
__global__ void givens_kernel(int R, int m, int j, const double2* __restrict__ hc, int hstride,
                              const double2* __restrict__ hn, double2* __restrict__ H, double2* __restrict__ cs,
                              double2* __restrict__ sn, double2* __restrict__ g, double* __restrict__ res,
                              int* __restrict__ jdone, const double* __restrict__ tol) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  if (jdone[r] >= 0) return;  // frozen: converged earlier in this cycle
  double2* Hr = H + (size_t)r * (m + 1) * m;
  double2* c = cs + (size_t)r * m;
  double2* s = sn + (size_t)r * m;
  double2* gr = g + (size_t)r * (m + 1);
  auto at = [&](int i) -> double2& { return Hr[(size_t)i * m + j]; };
  for (int i = 0; i <= j; ++i) at(i) = hc[(size_t)r * hstride + i];
  at(j + 1) = hn[(size_t)r * hstride];
  for (int i = 0; i < j; ++i) {
    const double2 a = at(i), b = at(i + 1);
    const double2 t = cadd<double>(cmul<double>(cconj<double>(c[i]), a), cmul<double>(cconj<double>(s[i]), b));
    at(i + 1) = csub<double>(cmul<double>(c[i], b), cmul<double>(s[i], a));
    at(i) = t;
  }
  const double2 a = at(j), b = at(j + 1);
  const double den = sqrt(a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y);
  if (den > 0) {
    c[j] = make_double2(a.x / den, a.y / den);
    s[j] = make_double2(b.x / den, b.y / den);
  } else {
    c[j] = make_double2(1, 0);
    s[j] = make_double2(0, 0);
  }
  at(j) = make_double2(den, 0.0);
  at(j + 1) = make_double2(0, 0);
  const double2 gj = gr[j];
  gr[j + 1] = csub<double>(make_double2(0, 0), cmul<double>(s[j], gj));
  gr[j] = cmul<double>(cconj<double>(c[j]), gj);
  const double e = sqrt(gr[j + 1].x * gr[j + 1].x + gr[j + 1].y * gr[j + 1].y);
  res[r] = e;
  if (e <= tol[r] || den == 0.0 || hn[(size_t)r * hstride].x == 0.0) jdone[r] = j + 1;
}

// y = H^{-1} g (upper triangular, size jd[r]); one thread per RHS
__global__ void backsolve_kernel(int R, int m, int jcur, const double2* __restrict__ H, const double2* __restrict__ g,
                                 const int* __restrict__ jdone, double2* __restrict__ y, int ystride) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int J = jdone[r] >= 0 ? jdone[r] : jcur;
  const double2* Hr = H + (size_t)r * (m + 1) * m;
  double2* yr = y + (size_t)r * ystride;
  for (int i = 0; i < ystride; ++i) yr[i] = make_double2(0, 0);
  for (int i = J - 1; i >= 0; --i) {
    double2 acc = g[(size_t)r * (m + 1) + i];
    for (int t = i + 1; t < J; ++t) acc = csub<double>(acc, cmul<double>(Hr[(size_t)i * m + t], yr[t]));
    const double2 d = Hr[(size_t)i * m + i];
    const double dd = d.x * d.x + d.y * d.y;
    yr[i] = dd > 0 ? make_double2((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd)
                   : make_double2(0, 0);
  }
}

// g = [beta, 0, ...], jdone = -1 (beta from the .x of hn)
__global__ void gmres_init_kernel(int R, int m, const double2* __restrict__ beta, double2* __restrict__ g,
                                  int* __restrict__ jdone) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  for (int i = 0; i <= m; ++i) g[(size_t)r * (m + 1) + i] = make_double2(0, 0);
  g[(size_t)r * (m + 1)] = make_double2(beta[r].x, 0);
  jdone[r] = beta[r].x > 0 ? -1 : 0;
}

struct Solver {
  const Plan& P;
  hipStream_t s;
  int R, m;
  size_t N;       // DOFs per RHS
  size_t vlen;    // R * N
  int nblk;
  std::vector<void*> mem;
  double2 *V = nullptr, *w = nullptr, *r = nullptr, *d = nullptr, *t = nullptr, *rin = nullptr;
  float2 *x32 = nullptr, *y32 = nullptr;
  void* ws = nullptr;
  double2 *part = nullptr, *hc = nullptr, *hn = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr,
          *y = nullptr;
  double *res = nullptr, *tol = nullptr;
  int* jdone = nullptr;
  int hstride;

  Solver(const Plan& p_, hipStream_t s_, int R_, int m_) : P(p_), s(s_), R(R_), m(m_) {
    N = (size_t)P.n * P.C;
    vlen = (size_t)R * N;
    nblk = (int)((N + kDotThreads * kEl - 1) / (kDotThreads * kEl));
    hstride = m + 2;
  }
  ~Solver() {
    for (void* q : mem) hipFree(q);
  }
  hipError_t alloc(void** q, size_t bytes) {
    hipError_t e = hipMalloc(q, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) mem.push_back(*q);
    return e;
  }
  hipError_t setup(bool need32) {
    hipError_t e;
    if ((e = alloc((void**)&V, (size_t)(m + 1) * vlen * sizeof(double2)))) return e;
    if ((e = alloc((void**)&w, vlen * sizeof(double2)))) return e;
    if ((e = alloc((void**)&r, vlen * sizeof(double2)))) return e;
    if ((e = alloc((void**)&d, vlen * sizeof(double2)))) return e;
    if ((e = alloc((void**)&t, vlen * sizeof(double2)))) return e;
    if (need32) {
      if ((e = alloc((void**)&rin, vlen * sizeof(double2)))) return e;
      if ((e = alloc((void**)&x32, vlen * sizeof(float2)))) return e;
      if ((e = alloc((void**)&y32, vlen * sizeof(float2)))) return e;
    }
    const size_t wsb = (size_t)R * std::max(matvec_workspace_bytes_per_rhs(P, 0), matvec_workspace_bytes_per_rhs(P, 1));
    if ((e = alloc(&ws, wsb))) return e;
    if ((e = alloc((void**)&part, (size_t)R * (m + 1) * nblk * sizeof(double2)))) return e;
    if ((e = alloc((void**)&hc, (size_t)R * hstride * sizeof(double2)))) return e;
    if ((e = alloc((void**)&hn, (size_t)R * hstride * sizeof(double2)))) return e;
    if ((e = alloc((void**)&H, (size_t)R * (m + 1) * m * sizeof(double2)))) return e;
    if ((e = alloc((void**)&cs, (size_t)R * m * sizeof(double2)))) return e;
    if ((e = alloc((void**)&sn, (size_t)R * m * sizeof(double2)))) return e;
    if ((e = alloc((void**)&g, (size_t)R * (m + 1) * sizeof(double2)))) return e;
    if ((e = alloc((void**)&y, (size_t)R * hstride * sizeof(double2)))) return e;
    if ((e = alloc((void**)&res, R * sizeof(double)))) return e;
    if ((e = alloc((void**)&tol, R * sizeof(double)))) return e;
    if ((e = alloc((void**)&jdone, R * sizeof(int)))) return e;
    return hipSuccess;
  }
  dim3 vgrid() const { return dim3((unsigned)std::min<size_t>((N + 255) / 256, 2048), R); }
  // out = A in (FP64 vectors); prec selects the operator copy
  hipError_t apply(int prec, const double2* in, double2* out) {
    if (prec == FMBEM_FP64) return matvec_launch(P, FMBEM_FP64, R, in, out, ws, s);
    const unsigned bl = (unsigned)std::min<size_t>((vlen + 255) / 256, 4096);
    hipLaunchKernelGGL(to32_kernel, dim3(bl), dim3(256), 0, s, in, x32, vlen);
    hipError_t e = matvec_launch(P, FMBEM_FP32, R, x32, y32, ws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(to64_kernel, dim3(bl), dim3(256), 0, s, y32, out, vlen);
    return hipGetLastError();
  }
  // dots of the first J basis vectors with vec -> h (mode 0 set / 1 add)
  void mdot(const double2* Vb, int J, const double2* vec, double2* h, int mode) {
    hipLaunchKernelGGL(mdot_kernel, dim3(nblk, R), dim3(kDotThreads), 0, s, Vb, vlen, vec, N, R, J, part);
    hipLaunchKernelGGL(mdot_finish, dim3((R * J + 127) / 128), dim3(128), 0, s, part, nblk, R, J, h, hstride, mode);
  }
  // per-RHS 2-norm of vec into hn[r][0]
  void norm(const double2* vec, double2* out) {
    hipLaunchKernelGGL(mdot_kernel, dim3(nblk, R), dim3(kDotThreads), 0, s, vec, vlen, vec, N, R, 1, part);
    hipLaunchKernelGGL(mdot_finish, dim3((R + 127) / 128), dim3(128), 0, s, part, nblk, R, 1, out, hstride, 2);
  }
  void maxpy(const double2* Vb, const double2* c, double2* vec, int J, double sgn) {
    hipLaunchKernelGGL(maxpy_kernel, vgrid(), dim3(256), J * sizeof(double2), s, Vb, vlen, c, hstride, vec, N, R, J,
                       sgn);
  }

  // Restarted GMRES on A_prec sol = rhs; sol is updated in place.  Stops per RHS
  // when the residual estimate drops below tol_abs[r]; returns iterations done.
  hipError_t gmres(int prec, const double2* rhs, double2* sol, const std::vector<double>& tol_abs, int max_its,
                   int& its, std::vector<double>& est) {
    hipError_t e = hipMemcpyAsync(tol, tol_abs.data(), R * sizeof(double), hipMemcpyHostToDevice, s);
    if (e) return e;
    std::vector<double> hres(R);
    std::vector<int> hj(R);
    est.assign(R, 0.0);
    while (true) {
      // r = rhs - A sol, beta = ||r||
      if ((e = apply(prec, sol, t))) return e;
      hipLaunchKernelGGL(sub_kernel, dim3(2048), dim3(256), 0, s, rhs, t, r, vlen);
      norm(r, hn);
      hipLaunchKernelGGL(gmres_init_kernel, dim3((R + 63) / 64), dim3(64), 0, s, R, m, hn, g, jdone);
      hipLaunchKernelGGL(scale_kernel, vgrid(), dim3(256), 0, s, r, hn, hstride, V, N, R, 1);
      std::vector<double2> hb(R * hstride);
      if ((e = hipMemcpyAsync(hb.data(), hn, R * hstride * sizeof(double2), hipMemcpyDeviceToHost, s))) return e;
      if ((e = hipStreamSynchronize(s))) return e;
      bool all = true;
      for (int q = 0; q < R; ++q) {
        est[q] = hb[(size_t)q * hstride].x;
        if (est[q] > tol_abs[q]) all = false;
      }
      if (all || its >= max_its) return hipSuccess;
      int j = 0;
      for (; j < m && its < max_its; ++j) {
        double2* vj = V + (size_t)j * vlen;
        if ((e = apply(prec, vj, w))) return e;
        // CGS2
        mdot(V, j + 1, w, hc, 0);
        maxpy(V, hc, w, j + 1, -1.0);
        mdot(V, j + 1, w, y, 0);
        maxpy(V, y, w, j + 1, -1.0);
        hipLaunchKernelGGL(add_kernel, dim3((R * hstride + 255) / 256), dim3(256), 0, s, hc, y,
                           (size_t)R * hstride);
        norm(w, hn);
        hipLaunchKernelGGL(givens_kernel, dim3((R + 63) / 64), dim3(64), 0, s, R, m, j, hc, hstride, hn, H, cs, sn,
                           g, res, jdone, tol);
        hipLaunchKernelGGL(scale_kernel, vgrid(), dim3(256), 0, s, w, hn, hstride, V + (size_t)(j + 1) * vlen, N, R,
                           1);
        ++its;
        if ((e = hipMemcpyAsync(hj.data(), jdone, R * sizeof(int), hipMemcpyDeviceToHost, s))) return e;
        if ((e = hipMemcpyAsync(hres.data(), res, R * sizeof(double), hipMemcpyDeviceToHost, s))) return e;
        if ((e = hipStreamSynchronize(s))) return e;
        bool done = true;
        for (int q = 0; q < R; ++q) {
          est[q] = hres[q];
          if (hj[q] < 0) done = false;
        }
        if (done) { ++j; break; }
      }
      // sol += V y
      hipLaunchKernelGGL(backsolve_kernel, dim3((R + 63) / 64), dim3(64), 0, s, R, m, j, H, g, jdone, y, hstride);
      maxpy(V, y, sol, m, 1.0);
      if ((e = hipGetLastError())) return e;
    }
  }
};

static fmbem_status st_of(hipError_t e) {
  if (e == hipSuccess) return FMBEM_OK;
  return e == hipErrorOutOfMemory ? FMBEM_ERR_OUT_OF_MEMORY : FMBEM_ERR_DEVICE;
}

}  // namespace fmbem

using namespace fmbem;

extern "C" fmbem_status fmbem_solve(fmbem_plan plan, const fmbem_solve_opts* opts, int32_t n_rhs, const void* b,
                                    void* x, fmbem_solve_info* info, void* hip_stream) {
  if (!plan || !opts || !b || !x || n_rhs < 1) return FMBEM_ERR_INVALID_ARG;
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  if (!(opts->tol > 0.0) || !std::isfinite(opts->tol)) return FMBEM_ERR_INVALID_ARG;
  const int m = opts->restart == 0 ? 30 : opts->restart;
  if (m < 1 || m > 200) return FMBEM_ERR_INVALID_ARG;
  const int max_its = opts->max_iters == 0 ? 1000 : opts->max_iters;
  const int max_ref = opts->max_refinements == 0 ? 20 : opts->max_refinements;
  const double inner_tol = opts->inner_tol == 0.0 ? 1e-5 : opts->inner_tol;
  if (max_its < 1 || max_ref < 1 || !(inner_tol > 0.0) || inner_tol >= 1.0) return FMBEM_ERR_INVALID_ARG;
  const int ip = opts->inner_precision;
  if (ip != FMBEM_FP64 && ip != FMBEM_FP32) return FMBEM_ERR_INVALID_ARG;
  if (!(P.precisions & 1u)) return FMBEM_ERR_UNSUPPORTED;  // the true residual needs the FP64 operator
  if (ip == FMBEM_FP32 && !(P.precisions & 2u)) return FMBEM_ERR_UNSUPPORTED;
  if ((size_t)n_rhs * P.C > (size_t)INT32_MAX / 2) return FMBEM_ERR_UNSUPPORTED;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  Solver S(P, s, n_rhs, m);
  hipError_t e = S.setup(ip == FMBEM_FP32);
  if (e) return st_of(e);
  const int R = n_rhs;
  const double2* bb = reinterpret_cast<const double2*>(b);
  double2* xx = reinterpret_cast<double2*>(x);
  // ||b||
  std::vector<double2> hb(R * S.hstride);
  S.norm(bb, S.hn);
  e = hipMemcpyAsync(hb.data(), S.hn, R * S.hstride * sizeof(double2), hipMemcpyDeviceToHost, s);
  if (!e) e = hipStreamSynchronize(s);
  if (e) return st_of(e);
  std::vector<double> bn(R), tabs(R);
  for (int q = 0; q < R; ++q) {
    bn[q] = hb[(size_t)q * S.hstride].x;
    if (!std::isfinite(bn[q])) return FMBEM_ERR_INVALID_ARG;
  }
  int its = 0, refs = 0;
  std::vector<double> est, rel(R, 0.0);
  auto true_residual = [&]() -> hipError_t {
    hipError_t ee = S.apply(FMBEM_FP64, xx, S.t);
    if (ee) return ee;
    hipLaunchKernelGGL(sub_kernel, dim3(2048), dim3(256), 0, s, bb, S.t, S.r, S.vlen);
    S.norm(S.r, S.hn);
    ee = hipMemcpyAsync(hb.data(), S.hn, R * S.hstride * sizeof(double2), hipMemcpyDeviceToHost, s);
    if (!ee) ee = hipStreamSynchronize(s);
    for (int q = 0; q < R; ++q) rel[q] = bn[q] > 0 ? hb[(size_t)q * S.hstride].x / bn[q] : 0.0;
    return ee;
  };
  bool ok = false;
  if (ip == FMBEM_FP64) {
    for (int q = 0; q < R; ++q) tabs[q] = opts->tol * bn[q];
    // GMRES estimates can drift from the true residual; re-enter while the true residual misses tol
    for (int rep = 0; rep < max_ref && !ok; ++rep) {
      e = S.gmres(FMBEM_FP64, bb, xx, tabs, max_its, its, est);
      if (e) return st_of(e);
      e = true_residual();
      if (e) return st_of(e);
      ok = true;
      for (int q = 0; q < R; ++q)
        if (!(rel[q] <= opts->tol)) ok = false;
      if (its >= max_its) break;
    }
  } else {
    for (refs = 0; refs < max_ref; ++refs) {
      e = true_residual();
      if (e) return st_of(e);
      ok = true;
      for (int q = 0; q < R; ++q)
        if (!(rel[q] <= opts->tol)) ok = false;
      if (ok || its >= max_its) break;
      // inner: A32 d = r, d0 = 0, to inner_tol * ||r|| (and not below what the outer needs)
      for (int q = 0; q < R; ++q) tabs[q] = std::max(inner_tol * rel[q] * bn[q], 0.5 * opts->tol * bn[q]);
      // the inner right-hand side lives in its own buffer: gmres() reuses r, t and w
      hipMemsetAsync(S.d, 0, S.vlen * sizeof(double2), s);
      hipMemcpyAsync(S.rin, S.r, S.vlen * sizeof(double2), hipMemcpyDeviceToDevice, s);
      e = S.gmres(FMBEM_FP32, S.rin, S.d, tabs, max_its, its, est);
      if (e) return st_of(e);
      hipLaunchKernelGGL(add_kernel, dim3(2048), dim3(256), 0, s, xx, S.d, S.vlen);
    }
  }
  if (info) {
    for (int q = 0; q < R; ++q) {
      info[q].iterations = its;
      info[q].refinements = refs;
      info[q].rel_residual = rel[q];
    }
  }
  return ok ? FMBEM_OK : FMBEM_ERR_NOT_CONVERGED;
}
