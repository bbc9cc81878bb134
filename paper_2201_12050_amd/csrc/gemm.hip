// Complex GEMM on the CDNA matrix cores, real-split form.
//
// C[:, j] (+)= sum_segments A_s B[:, col_s(j)]: A_s complex M x K row-major,
// B and C complex column-major with per-column address maps.  The same kernel
// carries the three dense contractions of the FMPBEM apply (Sec. 3.5, eq.
// (FMPBEMsystem)):
//   near field  y_c  = sum_{d in near} S_d x_{c-d}   (one segment per offset d)
//   S2M         m_c  = V0 x_c                        (written into the padded FFT grid)
//   L2T         y_c += U0 l_c                        (read from the padded FFT grid)
//
// A complex product is computed as the real product of the 2x2 split form
//   [Re A, -Im A; Im A, Re A] (2M x 2K)  x  [Re B; Im B] (2K x N)
// so that interleaved complex B columns are used as real columns of length 2K
// and the 16x16x4 MFMA tiles produce interleaved complex outputs.  A is read
// from HBM in complex form and expanded into the split form while it is staged
// into LDS.  Accumulation is in the operand precision.
#include "common.hpp"

namespace fmbem {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Output layout of the 16x16x4 tiles (checked on gfx950): lane l holds column l%16
// and four rows; for f32 these are rows 4g..4g+3, for f64 rows g, g+4, g+8, g+12
// (g = l/16).  rowpos() places the split-form row (complex row cr, component c)
// of a 16-row block so that every lane ends up holding (re, im) of complex rows
// 2g and 2g+1 in its accumulator registers (0, 1) and (2, 3), for both types.
template <typename T> struct mfma;
template <> struct mfma<double> {
  using acc = v4d;
  __device__ static inline int rowpos(int cr, int c) {
    const int blk = cr >> 3, cb = cr & 7;
    return 16 * blk + (cb >> 1) + 4 * (2 * (cb & 1) + c);
  }
  __device__ static inline acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct mfma<float> {
  using acc = v4f;
  __device__ static inline int rowpos(int cr, int c) { return 2 * cr + c; }
  __device__ static inline acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// column address map; returns nullptr for an all-zero column
template <typename T>
__device__ inline cplx<T>* col_ptr(const GemmCols& m, cplx<T>* base, int j, int d0, int d1, int d2) {
  if (m.kind == COL_LINEAR) return base + (size_t)j * m.ld;
  int r = j / m.C;
  int c = j - r * m.C;
  int i1 = c % m.g0;
  int t = c / m.g0;
  int i2 = t % m.g1;
  int i3 = t / m.g1;
  if (m.kind == COL_CELL_SHIFT) {
    int s1 = i1 - d0, s2 = i2 - d1, s3 = i3 - d2;
    if (s1 < 0 || s1 >= m.g0 || s2 < 0 || s2 >= m.g1 || s3 < 0 || s3 >= m.g2) return nullptr;
    int src = s1 + m.g0 * (s2 + m.g1 * s3);
    return base + ((size_t)r * m.C + src) * m.ld;
  }
  // COL_CELL_TO_BIN
  size_t bin = (size_t)i1 + (size_t)m.f0 * (i2 + (size_t)m.f1 * i3);
  return base + (bin * m.R + r) * m.ld;
}

constexpr int BMC = 32;           // complex rows per tile (64 real rows)
constexpr int BN = 64;            // columns per tile
constexpr int BKC = 8;            // complex k per step (16 real k)
constexpr int LDA = 2 * BMC + 4;  // padded LDS row (real rows)
constexpr int LDB = BN + 4;

template <typename T>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int K, int N, GemmSegs segs,
                                                   const cplx<T>* __restrict__ B, GemmCols bmap,
                                                   cplx<T>* __restrict__ Cm, GemmCols cmap,
                                                   int accumulate) {
  __shared__ T As[2 * BKC][LDA];
  __shared__ T Bs[2 * BKC][LDB];
  using Acc = typename mfma<T>::acc;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m0 = blockIdx.x * BMC;
  const int n0 = blockIdx.y * BN;
  const int wr = wave >> 1, wc = wave & 1;

  Acc acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = Acc{0, 0, 0, 0};

  // A staging: thread -> (row, kc)
  const int a_row = tid / BKC, a_kc = tid % BKC;
  // B staging: thread -> (col, kc pair)
  const int b_col = tid / 4, b_kc = (tid % 4) * 2;
  const int bj = n0 + b_col;

  for (int si = 0; si < segs.count; ++si) {
    const GemmSeg sg = segs.seg[si];
    const cplx<T>* A = reinterpret_cast<const cplx<T>*>(sg.A);
    const cplx<T>* bc = nullptr;
    if (bj < N) bc = col_ptr<T>(bmap, const_cast<cplx<T>*>(B), bj, sg.d0, sg.d1, sg.d2);
    for (int k0 = 0; k0 < K; k0 += BKC) {
      cplx<T> a = mk<T>(0, 0);
      {
        int m = m0 + a_row, kk = k0 + a_kc;
        if (m < M && kk < K) a = A[(size_t)m * K + kk];
      }
      cplx<T> b0 = mk<T>(0, 0), b1 = mk<T>(0, 0);
      if (bc) {
        int kk = k0 + b_kc;
        if (kk < K) b0 = bc[kk];
        if (kk + 1 < K) b1 = bc[kk + 1];
      }
      __syncthreads();
      const int pr = mfma<T>::rowpos(a_row, 0), pi = mfma<T>::rowpos(a_row, 1);
      As[2 * a_kc][pr] = a.x;
      As[2 * a_kc + 1][pr] = -a.y;
      As[2 * a_kc][pi] = a.y;
      As[2 * a_kc + 1][pi] = a.x;
      Bs[2 * b_kc][b_col] = b0.x;
      Bs[2 * b_kc + 1][b_col] = b0.y;
      Bs[2 * b_kc + 2][b_col] = b1.x;
      Bs[2 * b_kc + 3][b_col] = b1.y;
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < 2 * BKC; ks += 4) {
        const int kr = ks + (lane >> 4);
        T af[2], bf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) af[i] = As[kr][32 * wr + 16 * i + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 2; ++j) bf[j] = Bs[kr][32 * wc + 16 * j + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = mfma<T>::step(af[i], bf[j], acc[i][j]);
      }
    }
  }

  // epilogue: lane holds (re, im) of complex rows 2g and 2g+1 of each 16x16 block (see rowpos)
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int col = n0 + 32 * wc + 16 * j + (lane & 15);
    if (col >= N) continue;
    cplx<T>* cc = col_ptr<T>(cmap, Cm, col, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int rr = 32 * wr + 16 * i + 4 * (lane >> 4);
      const int m = m0 + rr / 2;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (m + h < M) {
          cplx<T> v = mk<T>(acc[i][j][2 * h], acc[i][j][2 * h + 1]);
          if (accumulate) v = cadd<T>(v, cc[m + h]);
          cc[m + h] = v;
        }
      }
    }
  }
}

template <typename T>
hipError_t gemm_launch(int M, int K, int N, const GemmSegs& segs, const void* B, GemmCols bmap,
                       void* Cm, GemmCols cmap, bool accumulate, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((M + BMC - 1) / BMC, (N + BN - 1) / BN);
  hipLaunchKernelGGL(gemm_kernel<T>, grid, dim3(256), 0, s, M, K, N, segs,
                     reinterpret_cast<const cplx<T>*>(B), bmap, reinterpret_cast<cplx<T>*>(Cm), cmap,
                     accumulate ? 1 : 0);
  return hipGetLastError();
}

template hipError_t gemm_launch<double>(int, int, int, const GemmSegs&, const void*, GemmCols, void*,
                                        GemmCols, bool, hipStream_t);
template hipError_t gemm_launch<float>(int, int, int, const GemmSegs&, const void*, GemmCols, void*,
                                       GemmCols, bool, hipStream_t);

}  // namespace fmbem
