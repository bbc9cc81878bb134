// Per-bin M2L product of the diagonalised far field (Sec. 2.4, eq. (diagonalized);
// Sec. 3.5, eq. (FMPBEMsystem)):  lhat_b = Lambda_b mhat_b  for every FFT bin b.
//
// HBM-bound for one right-hand side: Lambda (Bc p^2 complex, one matrix per pair of
// bins w, -w) is streamed once.  Lambda is stored column-major with an even column
// stride ldp, so that two consecutive rows form one aligned 16-byte (FP32) / 32-byte
// (FP64) load.  A workgroup owns one canonical bin and applies its matrix to the R
// vectors of the bin and the R vectors of its partner (whose spectrum carries the
// factor D of the symmetry, see grid_dft_launch): G groups of RP threads split the
// columns j, each thread of a group accumulates two rows for up to kRhs vectors, and
// the groups are summed in LDS.  The product is in place in the [bin][R][p] spectrum
// buffer.  FP32 takes 8 groups (twice the loads in flight of 4: a bin's matrix is only
// 118 KB at n_t = 10, measured 17.7 -> 13.7 us on 514 bins), FP64 4.  Measured and not kept
// (16x16 lattice, n_t = 10, inside the FP32-refined solve, 20.2 us): a bin's rows split over 2
// or 4 workgroups (20.4 / 21.4 us), and every matrix load of a thread issued before the vectors
// are staged (20.7 us).
#include <algorithm>
#include <vector>

#include "common.hpp"

namespace fmbem {

constexpr int kRhs = 4;
template <typename T> constexpr int gemv_groups() { return sizeof(T) == 4 ? 8 : 4; }

template <typename T> struct Pair;
template <> struct Pair<float> { using type = float4; };
template <> struct Pair<double> { using type = double4; };

// vector t of the pair (bin a: t < R, partner: t >= R) in the spectrum buffer
template <typename T>
__device__ inline cplx<T>* pair_vec(cplx<T>* buf, int a, int b, int R, int p, int t) {
  return buf + ((size_t)(t < R ? a : b) * R + (t < R ? t : t - R)) * p;
}

// several plans' products in one launch: workgroup blockIdx.x belongs to the last job whose block0
// it reaches and handles canonical bin blockIdx.x - block0 of that plan
struct M2lJob {
  const void* Lam;
  const int* pairs;
  void* buf;
  int R, p, ldp, block0;
};
constexpr int kMaxM2lJobs = 32;
struct M2lJobs {
  int count;
  M2lJob job[kMaxM2lJobs];
};

// RP row-pair threads per column group (p <= 2 RP) and G groups: RP * G threads
template <typename T, int RP, int G>
__global__ __launch_bounds__(RP * G) void m2l_gemv_kernel(M2lJobs J) {
  extern __shared__ unsigned char smem_raw[];
  int jq = 0;
  while (jq + 1 < J.count && (int)blockIdx.x >= J.job[jq + 1].block0) ++jq;
  const cplx<T>* __restrict__ Lam = reinterpret_cast<const cplx<T>*>(J.job[jq].Lam);
  const int* __restrict__ pairs = J.job[jq].pairs;
  cplx<T>* __restrict__ buf = reinterpret_cast<cplx<T>*>(J.job[jq].buf);
  const int R = J.job[jq].R, p = J.job[jq].p, ldp = J.job[jq].ldp;
  cplx<T>* xs = reinterpret_cast<cplx<T>*>(smem_raw);        // [kRhs][p]
  cplx<T>* red = xs + kRhs * p;                               // [G][RP][kRhs][2]
  using P2 = typename Pair<T>::type;
  const int c = (int)blockIdx.x - J.job[jq].block0;
  const int ba = pairs[2 * c], bb = pairs[2 * c + 1];
  const int nv = bb >= 0 ? 2 * R : R;
  const cplx<T>* Lb = Lam + (size_t)c * p * ldp;
  const int g = threadIdx.x / RP;
  const int rp = threadIdx.x % RP;                 // row pair (rows 2rp, 2rp+1)
  const int jc = (p + G - 1) / G;
  const int j0 = g * jc, j1 = min(p, j0 + jc);
  const bool active = 2 * rp < p;
  for (int r0 = 0; r0 < nv; r0 += kRhs) {
    const int nr = min(kRhs, nv - r0);
    __syncthreads();
    for (int t = threadIdx.x; t < nr * p; t += blockDim.x)
      xs[t] = pair_vec<T>(buf, ba, bb, R, p, r0 + t / p)[t % p];
    __syncthreads();
    cplx<T> a0[kRhs], a1[kRhs];
#pragma unroll
    for (int r = 0; r < kRhs; ++r) {
      a0[r] = mk<T>(0, 0);
      a1[r] = mk<T>(0, 0);
    }
    if (active) {
      const P2* col = reinterpret_cast<const P2*>(Lb + 2 * rp);
      const int step = ldp / 2;
#pragma unroll 4
      for (int j = j0; j < j1; ++j) {
        const P2 v = col[(size_t)j * step];
        const cplx<T> l0 = mk<T>(v.x, v.y), l1 = mk<T>(v.z, v.w);
#pragma unroll
        for (int r = 0; r < kRhs; ++r) {
          if (r < nr) {
            const cplx<T> m = xs[r * p + j];
            cfma<T>(a0[r], l0, m);
            cfma<T>(a1[r], l1, m);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kRhs; ++r) {
      red[((g * RP + rp) * kRhs + r) * 2] = a0[r];
      red[((g * RP + rp) * kRhs + r) * 2 + 1] = a1[r];
    }
    __syncthreads();
    if (g == 0 && active) {
#pragma unroll
      for (int r = 0; r < kRhs; ++r) {
        if (r < nr) {
          cplx<T> s0 = red[(rp * kRhs + r) * 2], s1 = red[(rp * kRhs + r) * 2 + 1];
          for (int q = 1; q < G; ++q) {
            s0 = cadd<T>(s0, red[((q * RP + rp) * kRhs + r) * 2]);
            s1 = cadd<T>(s1, red[((q * RP + rp) * kRhs + r) * 2 + 1]);
          }
          cplx<T>* out = pair_vec<T>(buf, ba, bb, R, p, r0 + r);
          out[2 * rp] = s0;
          if (2 * rp + 1 < p) out[2 * rp + 1] = s1;
        }
      }
    }
  }
}

// generic fallback for p > 256 (n_t >= 16, exact PBEM blocks): one thread per row
template <typename T>
__global__ void m2l_rows_kernel(M2lJobs J) {
  extern __shared__ unsigned char smem_raw[];
  int jq = 0;
  while (jq + 1 < J.count && (int)blockIdx.x >= J.job[jq + 1].block0) ++jq;
  const cplx<T>* __restrict__ Lam = reinterpret_cast<const cplx<T>*>(J.job[jq].Lam);
  const int* __restrict__ pairs = J.job[jq].pairs;
  cplx<T>* __restrict__ buf = reinterpret_cast<cplx<T>*>(J.job[jq].buf);
  const int R = J.job[jq].R, p = J.job[jq].p, ldp = J.job[jq].ldp;
  cplx<T>* xs = reinterpret_cast<cplx<T>*>(smem_raw);  // [kRhs][p]
  const int c = (int)blockIdx.x - J.job[jq].block0;
  const int ba = pairs[2 * c], bb = pairs[2 * c + 1];
  const int nv = bb >= 0 ? 2 * R : R;
  const cplx<T>* Lb = Lam + (size_t)c * p * ldp;
  for (int r0 = 0; r0 < nv; r0 += kRhs) {
    const int nr = min(kRhs, nv - r0);
    __syncthreads();
    for (int t = threadIdx.x; t < nr * p; t += blockDim.x)
      xs[t] = pair_vec<T>(buf, ba, bb, R, p, r0 + t / p)[t % p];
    __syncthreads();
    for (int i = threadIdx.x; i < p; i += blockDim.x) {
      cplx<T> acc[kRhs];
#pragma unroll
      for (int r = 0; r < kRhs; ++r) acc[r] = mk<T>(0, 0);
      for (int j = 0; j < p; ++j) {
        const cplx<T> a = Lb[(size_t)j * ldp + i];
#pragma unroll
        for (int r = 0; r < kRhs; ++r)
          if (r < nr) cfma<T>(acc[r], a, xs[r * p + j]);
      }
#pragma unroll
      for (int r = 0; r < kRhs; ++r)
        if (r < nr) pair_vec<T>(buf, ba, bb, R, p, r0 + r)[i] = acc[r];
    }
  }
}

int lambda_ld(int p) { return p + (p & 1); }

// kernel form of a plan's product: 0 the GEMV with 64 row pairs (p <= 128), 1 with 128 row pairs
// (p <= 256), 2 one thread per row
static int m2l_form(int p) { return p <= 128 ? 0 : (p <= 256 ? 1 : 2); }

template <typename T>
static hipError_t m2l_launch_form(int form, const std::vector<M2lProduct>& v, hipStream_t s) {
  for (size_t i0 = 0; i0 < v.size(); i0 += kMaxM2lJobs) {
    M2lJobs J{};
    int blocks = 0, pmax = 1;
    for (size_t i = i0; i < std::min(v.size(), i0 + kMaxM2lJobs); ++i) {
      M2lJob& j = J.job[J.count++];
      j.Lam = v[i].Lam;
      j.pairs = v[i].pairs;
      j.buf = v[i].buf;
      j.R = v[i].R;
      j.p = v[i].p;
      j.ldp = lambda_ld(v[i].p);
      j.block0 = blocks;
      blocks += v[i].Bc;
      pmax = std::max(pmax, v[i].p);
    }
    if (form == 0) {
      constexpr int G = gemv_groups<T>();
      const size_t lds = (size_t)(kRhs * pmax + G * 64 * kRhs * 2) * sizeof(cplx<T>);
      hipLaunchKernelGGL((m2l_gemv_kernel<T, 64, G>), dim3(blocks), dim3(64 * G), lds, s, J);
    } else if (form == 1) {
      const size_t lds = (size_t)(kRhs * pmax + 4 * 128 * kRhs * 2) * sizeof(cplx<T>);
      hipLaunchKernelGGL((m2l_gemv_kernel<T, 128, 4>), dim3(blocks), dim3(128 * 4), lds, s, J);
    } else {
      const int threads = std::min(512, ((pmax + 63) / 64) * 64);
      hipLaunchKernelGGL(m2l_rows_kernel<T>, dim3(blocks), dim3(threads), kRhs * pmax * sizeof(cplx<T>), s, J);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// the GEMV products of several plans, one launch per kernel form
template <typename T>
hipError_t m2l_group_launch(const std::vector<M2lProduct>& v, hipStream_t s) {
  for (int form = 0; form < 3; ++form) {
    std::vector<M2lProduct> sel;
    for (const M2lProduct& q : v)
      if (m2l_form(q.p) == form) sel.push_back(q);
    if (sel.empty()) continue;
    const hipError_t e = m2l_launch_form<T>(form, sel, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t m2l_launch(const void* Lam, const int* pairs, int Bc, void* buf, int R, int p, hipStream_t s) {
  return m2l_group_launch<T>({M2lProduct{Lam, pairs, Bc, buf, R, p}}, s);
}

template hipError_t m2l_launch<double>(const void*, const int*, int, void*, int, int, hipStream_t);
template hipError_t m2l_launch<float>(const void*, const int*, int, void*, int, int, hipStream_t);
template hipError_t m2l_group_launch<double>(const std::vector<M2lProduct>&, hipStream_t);
template hipError_t m2l_group_launch<float>(const std::vector<M2lProduct>&, hipStream_t);

}  // namespace fmbem
