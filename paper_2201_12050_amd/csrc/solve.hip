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
#include <cmath>
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

// part[r][i][blk] = sum_{n in block} conj(V_i[r][n]) w[r][n]; grid (blocks, vector groups of 8, R)
__global__ __launch_bounds__(kDotThreads) void mdot_kernel(const double2* __restrict__ V, size_t vstride,
                                                           const double2* __restrict__ w, size_t N, int J,
                                                           double2* __restrict__ part, const int* __restrict__ flag) {
  __shared__ double2 red[kDotThreads / 64][kDotVec];
  const int r = blockIdx.z;
  if (flag && !flag[r]) return;  // conditional pass not needed for this RHS
  const int i0 = blockIdx.y * kDotVec;
  const int nblk = gridDim.x;
  const size_t base = (size_t)blockIdx.x * kDotThreads * kDotEl + threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double2 wl[kDotEl];
#pragma unroll
  for (int e = 0; e < kDotEl; ++e) {
    const size_t n = base + (size_t)e * kDotThreads;
    wl[e] = n < N ? w[(size_t)r * N + n] : make_double2(0, 0);
  }
  double2 acc[kDotVec];
#pragma unroll
  for (int q = 0; q < kDotVec; ++q) {
    acc[q] = make_double2(0, 0);
    if (i0 + q < J) {
      const double2* vi = V + (size_t)(i0 + q) * vstride + (size_t)r * N;
#pragma unroll
      for (int e = 0; e < kDotEl; ++e) {
        const size_t n = base + (size_t)e * kDotThreads;
        if (n < N) {
          const double2 a = vi[n];
          acc[q].x += a.x * wl[e].x + a.y * wl[e].y;
          acc[q].y += a.x * wl[e].y - a.y * wl[e].x;
        }
      }
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
    part[((size_t)r * J + i0 + threadIdx.x) * nblk + blockIdx.x] = s;
  }
}

// one wave per (r, i) sums the block partials s; mode 0: h = s; mode 2: h = sqrt(Re s);
// mode 3: h2 = s and h += s (second Gram-Schmidt pass)
__global__ void mdot_finish(const double2* __restrict__ part, int nblk, int R, int J, double2* __restrict__ h,
                            int hstride, int mode, double2* __restrict__ h2, const int* __restrict__ flag) {
  const int t = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
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
  else if (mode == 2) *o = make_double2(sqrt(fmax(sx, 0.0)), 0.0);
  else {
    h2[(size_t)r * hstride + i] = make_double2(sx, sy);
    o->x += sx;
    o->y += sy;
  }
}

// w[r][n] += sgn * sum_{i<J} c[r][i] V_i[r][n]; with npart, also per-block sums of |w|^2
__global__ __launch_bounds__(256) void maxpy_kernel(const double2* __restrict__ V, size_t vstride,
                                                    const double2* __restrict__ c, int cstride,
                                                    double2* __restrict__ w, size_t N, int J, double sgn,
                                                    double* __restrict__ npart, const int* __restrict__ flag) {
  extern __shared__ double2 cs[];
  __shared__ double red[4];
  const int r = blockIdx.y;
  if (flag && !flag[r]) return;
  for (int i = threadIdx.x; i < J; i += blockDim.x) cs[i] = c[(size_t)r * cstride + i];
  __syncthreads();
  double nn = 0.0;
  for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (size_t)gridDim.x * blockDim.x) {
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
    if (threadIdx.x == 0) npart[(size_t)r * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
  }
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

// One workgroup per RHS: hn = sqrt(sum of the |w|^2 block partials), then the Givens
// update of Hessenberg column j (rotations [[conj(c), conj(s)], [-s, c]]) and of g on
// LDS copies, the residual estimate |g_{j+1}| and the freeze flag (also written to
// mapped host memory for the host's convergence check).
constexpr int kMaxRestart = 200;
__global__ __launch_bounds__(256) void norm_givens_kernel(const double* __restrict__ npart, int nb, int m, int j,
                                                          const double2* __restrict__ hc, int hstride,
                                                          double2* __restrict__ hn, double2* __restrict__ H,
                                                          double2* __restrict__ cs, double2* __restrict__ sn,
                                                          double2* __restrict__ g, double* __restrict__ res,
                                                          int* __restrict__ jdone, int* __restrict__ jdone_host,
                                                          const double* __restrict__ tol) {
  __shared__ double2 col[kMaxRestart + 2], lc[kMaxRestart], ls[kMaxRestart];
  __shared__ double red[4];
  const int r = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += npart[(size_t)r * nb + b];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double nrm = sqrt(fmax(red[0] + red[1] + red[2] + red[3], 0.0));
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

// y = H^{-1} g (upper triangular, size jdone[r] or jcur) by column sweeps; one workgroup per RHS
__global__ __launch_bounds__(256) void backsolve_kernel(int m, int jcur, const double2* __restrict__ H,
                                                        const double2* __restrict__ g,
                                                        const int* __restrict__ jdone, double2* __restrict__ y,
                                                        int ystride) {
  __shared__ double2 gl[kMaxRestart + 1];
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

struct Solver {
  const Plan& P;
  hipStream_t s;
  int R, m;
  int ortho = 0;  // FMBEM_ORTHO_*
  size_t N;       // DOFs per RHS
  size_t vlen;    // R * N
  int nblk;
  std::vector<void*> mem;
  double2 *V = nullptr, *w = nullptr, *r = nullptr, *d = nullptr, *t = nullptr, *rin = nullptr;
  float2 *x32 = nullptr, *y32 = nullptr;
  void* ws = nullptr;
  double2 *part = nullptr, *hc = nullptr, *hn = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr,
          *y = nullptr;
  double *res = nullptr, *tol = nullptr, *npart = nullptr;
  int* jdone = nullptr;
  int* reorth = nullptr;  // per-RHS second Gram-Schmidt pass flag
  // freeze flags of two steps in flight, in mapped pinned host memory written by the device
  int* hjd[2] = {nullptr, nullptr};
  int* djd[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  int hstride;
  int nb;  // workgroups of the multi-axpy kernel (and of its norm partials)

  Solver(const Plan& p_, hipStream_t s_, int R_, int m_) : P(p_), s(s_), R(R_), m(m_) {
    N = (size_t)P.n * P.C;
    vlen = (size_t)R * N;
    nblk = (int)((N + kDotThreads * kDotEl - 1) / (kDotThreads * kDotEl));
    hstride = m + 2;
    nb = (int)std::min<size_t>((N + 255) / 256, 2048);
  }
  ~Solver() {
    for (void* q : mem) hipFree(q);
    for (int i = 0; i < 2; ++i) {
      if (hjd[i]) hipHostFree(hjd[i]);
      if (ev[i]) hipEventDestroy(ev[i]);
    }
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
    if ((e = alloc((void**)&rin, vlen * sizeof(double2)))) return e;
    if (need32) {
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
    if ((e = alloc((void**)&npart, (size_t)R * nb * sizeof(double)))) return e;
    if ((e = alloc((void**)&reorth, R * sizeof(int)))) return e;
    for (int i = 0; i < 2; ++i) {
      if ((e = hipHostMalloc((void**)&hjd[i], R * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent)))
        return e;
      if ((e = hipHostGetDevicePointer((void**)&djd[i], hjd[i], 0))) return e;
      if ((e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming))) return e;
    }
    return hipSuccess;
  }
  dim3 vgrid() const { return dim3((unsigned)nb, R); }
  unsigned lgrid(size_t len) const { return (unsigned)std::min<size_t>((len + 255) / 256, 4096); }
  // out = A in (FP64 vectors); prec selects the operator copy; in32 (optional) = in already cast
  hipError_t apply(int prec, const double2* in, double2* out, const float2* in32 = nullptr) {
    if (prec == FMBEM_FP64) return matvec_launch(P, FMBEM_FP64, R, in, out, ws, s);
    if (!in32) {
      hipLaunchKernelGGL(to32_kernel, dim3(lgrid(vlen)), dim3(256), 0, s, in, x32, vlen);
      in32 = x32;
    }
    // the FP32 operator writes its result directly as FP64 into out
    return matvec_launch(P, FMBEM_FP32, R, in32, y32, ws, s, out);
  }
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

  // Restarted GMRES on A_prec sol = rhs; sol is updated in place.  Stops per RHS
  // when the residual estimate drops below tol_abs[r]; its counts operator applications
  // of the Arnoldi steps.
  hipError_t gmres(int prec, const double2* rhs, double2* sol, const std::vector<double>& tol_abs, int max_its,
                   int& its) {
    hipError_t e = hipMemcpyAsync(tol, tol_abs.data(), R * sizeof(double), hipMemcpyHostToDevice, s);
    if (e) return e;
    while (true) {
      // r = rhs - A sol, beta = ||r||, v_0 = r / beta
      if ((e = apply(prec, sol, t))) return e;
      hipLaunchKernelGGL(sub_kernel, dim3(lgrid(vlen)), dim3(256), 0, s, rhs, t, r, vlen);
      norm(r, hn);
      hipLaunchKernelGGL(gmres_init_kernel, dim3((R + 63) / 64), dim3(64), 0, s, R, m, hn, hstride, tol, g, jdone,
                         djd[0], res);
      hipLaunchKernelGGL(scale_kernel, vgrid(), dim3(256), 0, s, r, hn, hstride, V, prec == FMBEM_FP32 ? x32 : nullptr,
                         N);
      if ((e = hipStreamSynchronize(s))) return e;
      bool all = true;
      for (int q = 0; q < R; ++q)
        if (hjd[0][q] < 0) all = false;
      if (all || its >= max_its) return hipSuccess;
      int j = 0;
      int pending = -1;  // step whose freeze flags are in flight
      bool done = false;
      for (; j < m && its < max_its; ++j) {
        double2* vj = V + (size_t)j * vlen;
        double2* wv = V + (size_t)(j + 1) * vlen;  // w = A v_j is built in the slot of v_{j+1}
        // the FP32 copy of v_j was written by the scale kernel that produced it
        if ((e = apply(prec, vj, wv, prec == FMBEM_FP32 ? x32 : nullptr))) return e;
        // Gram-Schmidt: h = V^H w (and ||w||^2 as the last dot), w -= V h (with |w|^2 partials);
        // second pass h2 = V^H w, w -= V h2, h += h2 only where the DGKS criterion asks for it
        mdot(V, j + 2, wv, hc, 0);
        maxpy(V, hc, wv, j + 1, -1.0, true);
        hipLaunchKernelGGL(reorth_check_kernel, dim3(R), dim3(256), 0, s, ortho, nb, npart, hc, hstride, j, jdone,
                           reorth);
        mdot(V, j + 1, wv, hc, 3, y, reorth);
        maxpy(V, y, wv, j + 1, -1.0, true, reorth);
        const int slot = j & 1;
        hipLaunchKernelGGL(norm_givens_kernel, dim3(R), dim3(256), 0, s, npart, nb, m, j, hc, hstride, hn, H, cs, sn,
                           g, res, jdone, djd[slot], tol);
        hipLaunchKernelGGL(scale_kernel, vgrid(), dim3(256), 0, s, wv, hn, hstride, wv,
                           prec == FMBEM_FP32 ? x32 : nullptr, N);
        ++its;
        if ((e = hipEventRecord(ev[slot], s))) return e;
        // check the previous step while this one runs
        if (pending >= 0) {
          if ((e = hipEventSynchronize(ev[pending & 1]))) return e;
          done = true;
          for (int q = 0; q < R; ++q)
            if (hjd[pending & 1][q] < 0) done = false;
          if (done) {
            ++j;
            break;
          }
        }
        pending = j;
      }
      if (!done && pending >= 0) {
        // last step of the cycle: nothing left to overlap with
        if ((e = hipEventSynchronize(ev[pending & 1]))) return e;
      }
      // sol += V y
      hipLaunchKernelGGL(backsolve_kernel, dim3(R), dim3(256), 0, s, m, j, H, g, jdone, y, hstride);
      maxpy(V, y, sol, j, 1.0);  // y is zero beyond each RHS's own step count
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
  if (opts->orthogonalization < FMBEM_ORTHO_DGKS || opts->orthogonalization > FMBEM_ORTHO_ONCE)
    return FMBEM_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  Solver S(P, s, n_rhs, m);
  S.ortho = opts->orthogonalization;
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
  std::vector<double> rel(R, 0.0);
  auto true_residual = [&]() -> hipError_t {
    hipError_t ee = S.apply(FMBEM_FP64, xx, S.t);
    if (ee) return ee;
    hipLaunchKernelGGL(sub_kernel, dim3(S.lgrid(S.vlen)), dim3(256), 0, s, bb, S.t, S.r, S.vlen);
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
      e = S.gmres(FMBEM_FP64, bb, xx, tabs, max_its, its);
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
      // inner: A32 d = r, d0 = 0, to inner_tol * ||r|| (and not below what the outer needs);
      // the inner right-hand side lives in its own buffer since gmres() reuses r, t and w
      for (int q = 0; q < R; ++q) tabs[q] = std::max(inner_tol * rel[q] * bn[q], 0.5 * opts->tol * bn[q]);
      hipLaunchKernelGGL(zero_kernel, dim3(S.lgrid(S.vlen)), dim3(256), 0, s, S.d, S.vlen);
      hipLaunchKernelGGL(copy_kernel, dim3(S.lgrid(S.vlen)), dim3(256), 0, s, S.rin, S.r, S.vlen);
      e = S.gmres(FMBEM_FP32, S.rin, S.d, tabs, max_its, its);
      if (e) return st_of(e);
      hipLaunchKernelGGL(add_kernel, dim3(S.lgrid(S.vlen)), dim3(256), 0, s, xx, S.d, S.vlen);
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
