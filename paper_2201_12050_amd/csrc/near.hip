// Grouped complex GEMM on the matrix cores for the dense contractions of the
// FMPBEM apply (Sec. 3.2, eq. (2dPeriodicFMM); Sec. 3.5, eq. (FMPBEMsystem)):
//
//   near field  part_d[:, (r,c)] = S_d x_{(r, c-d)}   for every near offset d  (n x n blocks)
//   S2M         mhat[bin(c)][r]  = V0 x_{(r, c)}                                (p x n, into the padded grid)
//   L2T         y[:, (r,c)]      = sum_d part_d[:, (r,c)] + U0 l[bin(c)][r]     (n x p, from the padded grid)
//
// A job is one GEMM whose B columns are the cells (x right-hand sides) of x,
// shifted by the job's cell offset, or the bins of the padded grid.  A workgroup
// owns a tile of ROWS complex rows of one job and COLS columns, so the job's A
// tile is streamed from HBM once per column chunk while B stays in L2.  The near
// partial products are summed in a fixed order in the L2T epilogue
// (deterministic, independent of batching).
//
// Complex products use the real 2x2 split form [Re A, -Im A; Im A, Re A] x
// [Re B; Im B] on 16x16x4 MFMA tiles: A is read in complex form and expanded
// while staged into LDS, B columns are interleaved complex read as real columns
// of length 2K.  Global loads for the next K step are issued before the MFMAs of
// the current one.
#include <algorithm>

#include "common.hpp"

namespace fmbem {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Output layout of the 16x16x4 tiles (checked on gfx950): lane l holds column l%16
// and four rows; f32: rows 4g..4g+3, f64: rows g, g+4, g+8, g+12 (g = l/16).
// rowpos() places split-form row (complex row cr, component c) of a 16-row block so
// that every lane holds (re, im) of complex rows 2g, 2g+1 in registers (0,1), (2,3).
template <typename T> struct nmf;
template <> struct nmf<double> {
  using acc = v4d;
  __device__ static inline int rowpos(int cr, int c) {
    const int blk = cr >> 3, cb = cr & 7;
    return 16 * blk + (cb >> 1) + 4 * (2 * (cb & 1) + c);
  }
  __device__ static inline acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct nmf<float> {
  using acc = v4f;
  __device__ static inline int rowpos(int cr, int c) { return 2 * cr + c; }
  __device__ static inline acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

__device__ inline void cell_coords(const NearGrid& g, int j, int& r, int& i1, int& i2, int& i3) {
  r = j / g.C;
  const int c = j - r * g.C;
  i1 = c % g.M0;
  const int t = c / g.M0;
  i2 = t % g.M1;
  i3 = t / g.M1;
}

// Tile: ROWS complex rows x COLS columns, 4 waves arranged WR x (4/WR), KC complex k per step.
template <typename T, int ROWS, int COLS, int WR, int KC>
__device__ __forceinline__ void near_tile(int n, int N, const NearJobs& jobs, const cplx<T>* __restrict__ x,
                                          const cplx<T>* __restrict__ grid, const NearGrid& g) {
  constexpr int WC = 4 / WR;
  constexpr int RR = 2 * ROWS;          // real rows per tile
  constexpr int RBW = RR / (16 * WR);   // 16-row MFMA blocks per wave
  constexpr int CBW = COLS / (16 * WC); // 16-column MFMA blocks per wave
  static_assert(RBW >= 1 && CBW >= 1, "tile too small for the wave grid");
  constexpr int LDA = RR + 4;
  constexpr int LDB = COLS + 4;
  constexpr int BPT = COLS * KC / 256; // B complex elements per thread per step
  constexpr int TPC = KC / BPT;        // threads per column
  __shared__ T As[2 * KC][LDA];
  __shared__ T Bs[2 * KC][LDB];
  using Acc = typename nmf<T>::acc;

  // job lookup
  int ji = 0;
  while (ji + 1 < jobs.count && (int)blockIdx.x >= jobs.job[ji + 1].tile0) ++ji;
  const NearJob jb = jobs.job[ji];
  const int m0 = ((int)blockIdx.x - jb.tile0) * ROWS;
  const int M = jb.M, K = jb.K;
  const cplx<T>* A = reinterpret_cast<const cplx<T>*>(jb.A);
  const int col0 = blockIdx.y * COLS;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;

  // B column of this thread; nullptr = zero column (shifted outside the grid)
  const int b_col = tid / TPC;
  const int b_k = (tid % TPC) * BPT;
  const cplx<T>* bcol = nullptr;
  {
    const int j = col0 + b_col;
    if (j < N) {
      int r, i1, i2, i3;
      cell_coords(g, j, r, i1, i2, i3);
      if (jb.src == SRC_X) {
        const int s1 = i1 - jb.d0, s2 = i2 - jb.d1, s3 = i3 - jb.d2;
        if (s1 >= 0 && s1 < g.M0 && s2 >= 0 && s2 < g.M1 && s3 >= 0 && s3 < g.M2)
          bcol = x + ((size_t)r * g.C + (s1 + g.M0 * (s2 + g.M1 * s3))) * n;
      } else {
        const size_t bin = (size_t)i1 + (size_t)g.N0 * (i2 + (size_t)g.N1 * i3);
        bcol = grid + (bin * g.R + r) * K;
      }
    }
  }
  // A staging: ROWS x KC complex per step, APT per thread
  constexpr int AT = ROWS * KC;
  constexpr int APT = AT >= 256 ? AT / 256 : 1;

  Acc acc[RBW][CBW];
#pragma unroll
  for (int i = 0; i < RBW; ++i)
#pragma unroll
    for (int j = 0; j < CBW; ++j) acc[i][j] = Acc{0, 0, 0, 0};

  cplx<T> ra[APT];
  cplx<T> rb[BPT];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < APT; ++q) {
      ra[q] = mk<T>(0, 0);
      const int e = tid + 256 * q;
      if (e < AT) {
        const int m = m0 + e / KC, kk = k0 + e % KC;
        if (m < M && kk < K) ra[q] = A[(size_t)m * K + kk];
      }
    }
#pragma unroll
    for (int e = 0; e < BPT; ++e) rb[e] = mk<T>(0, 0);
    if (bcol) {
      if (k0 + KC <= K) {
#pragma unroll
        for (int e = 0; e < BPT; ++e) rb[e] = bcol[k0 + b_k + e];
      } else {
        for (int e = 0; e < BPT; ++e)
          if (k0 + b_k + e < K) rb[e] = bcol[k0 + b_k + e];
      }
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < APT; ++q) {
      const int e = tid + 256 * q;
      if (e < AT) {
        const int row = e / KC, kc = e % KC;
        const int pr = nmf<T>::rowpos(row, 0), pi = nmf<T>::rowpos(row, 1);
        As[2 * kc][pr] = ra[q].x;
        As[2 * kc + 1][pr] = -ra[q].y;
        As[2 * kc][pi] = ra[q].y;
        As[2 * kc + 1][pi] = ra[q].x;
      }
    }
#pragma unroll
    for (int e = 0; e < BPT; ++e) {
      Bs[2 * (b_k + e)][b_col] = rb[e].x;
      Bs[2 * (b_k + e) + 1][b_col] = rb[e].y;
    }
    __syncthreads();
    if (k0 + KC < K) load(k0 + KC);
#pragma unroll
    for (int ks = 0; ks < 2 * KC; ks += 4) {
      const int kr = ks + (lane >> 4);
      T af[RBW], bf[CBW];
#pragma unroll
      for (int i = 0; i < RBW; ++i) af[i] = As[kr][16 * (RBW * wr + i) + (lane & 15)];
#pragma unroll
      for (int j = 0; j < CBW; ++j) bf[j] = Bs[kr][16 * (CBW * wc + j) + (lane & 15)];
#pragma unroll
      for (int i = 0; i < RBW; ++i)
#pragma unroll
        for (int j = 0; j < CBW; ++j) acc[i][j] = nmf<T>::step(af[i], bf[j], acc[i][j]);
    }
  }

  // epilogue: (re, im) of complex rows 2g, 2g+1 of each 16-row block (see rowpos)
  cplx<T>* out = reinterpret_cast<cplx<T>*>(jb.out);
  const cplx<T>* part = reinterpret_cast<const cplx<T>*>(jb.part);
  double2* out64 = reinterpret_cast<double2*>(jb.out64);
  const size_t slice = (size_t)N * M;
#pragma unroll
  for (int j = 0; j < CBW; ++j) {
    const int col = col0 + 16 * (CBW * wc + j) + (lane & 15);
    if (col >= N) continue;
    size_t base;
    if (jb.dest == DEST_GRID) {
      int r, i1, i2, i3;
      cell_coords(g, col, r, i1, i2, i3);
      const size_t bin = (size_t)i1 + (size_t)g.N0 * (i2 + (size_t)g.N1 * i3);
      base = (bin * g.R + r) * M;
    } else {
      base = (size_t)col * M;
    }
#pragma unroll
    for (int i = 0; i < RBW; ++i) {
      const int m = m0 + 8 * (RBW * wr + i) + 2 * (lane >> 4);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (m + h >= M) continue;
        cplx<T> v = mk<T>(acc[i][j][2 * h], acc[i][j][2 * h + 1]);
        if (jb.dest == DEST_FINAL) {
          for (int q = 0; q < jb.nparts; ++q) v = cadd<T>(v, part[q * slice + base + m + h]);
          if (out64) {
            out64[base + m + h] = make_double2((double)v.x, (double)v.y);
            continue;
          }
        }
        out[base + m + h] = v;
      }
    }
  }
}

// The same tile body under two kernel names, so that per-kernel profiles keep the near-field/S2M
// launch apart from the L2T launch even when both use the same tile shape.
template <typename T, int ROWS, int COLS, int WR, int KC>
__global__ __launch_bounds__(256) void near_kernel(int n, int N, NearJobs jobs, const cplx<T>* __restrict__ x,
                                                   const cplx<T>* __restrict__ grid, NearGrid g) {
  near_tile<T, ROWS, COLS, WR, KC>(n, N, jobs, x, grid, g);
}
template <typename T, int ROWS, int COLS, int WR, int KC>
__global__ __launch_bounds__(256) void l2t_kernel(int n, int N, NearJobs jobs, const cplx<T>* __restrict__ x,
                                                  const cplx<T>* __restrict__ grid, NearGrid g) {
  near_tile<T, ROWS, COLS, WR, KC>(n, N, jobs, x, grid, g);
}

// y[col][m] = sum_s part[s][col][m] in a fixed order (optionally written as FP64)
template <typename T>
__global__ void near_reduce_kernel(const cplx<T>* __restrict__ part, int ns, size_t len, cplx<T>* __restrict__ y,
                                   double2* __restrict__ y64) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (size_t)gridDim.x * blockDim.x) {
    cplx<T> s = part[i];
    for (int q = 1; q < ns; ++q) s = cadd<T>(s, part[(size_t)q * len + i]);
    if (y64) y64[i] = make_double2((double)s.x, (double)s.y);
    else y[i] = s;
  }
}

// tile shapes: (complex rows, columns, wave rows, complex k per step)
struct NearShape {
  int rows, cols, wr, kc;
};
static const NearShape kShapes[] = {{16, 256, 1, 8}, {32, 256, 1, 8}, {32, 128, 2, 8},  {64, 64, 4, 8},
                                    {32, 64, 2, 8},  {16, 128, 1, 8}, {16, 64, 1, 8},   {32, 128, 2, 16},
                                    {64, 64, 4, 16}, {16, 128, 1, 16}, {64, 128, 2, 8}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

int near_num_shapes() { return kNumShapes; }

template <typename T, int ROWS, int COLS, int WR, int KC>
static void launch_shape(dim3 grid, hipStream_t s, int kind, int n, int N, const NearJobs& jobs, const void* x,
                         const void* gridbuf, const NearGrid& g) {
  const cplx<T>* xs = reinterpret_cast<const cplx<T>*>(x);
  const cplx<T>* gs = reinterpret_cast<const cplx<T>*>(gridbuf);
  if (kind == 1)
    hipLaunchKernelGGL((l2t_kernel<T, ROWS, COLS, WR, KC>), grid, dim3(256), 0, s, n, N, jobs, xs, gs, g);
  else
    hipLaunchKernelGGL((near_kernel<T, ROWS, COLS, WR, KC>), grid, dim3(256), 0, s, n, N, jobs, xs, gs, g);
}

// default shape: the one whose workgroup count best fills whole rounds of 256 CUs
static int near_default_shape(int N, const NearJobs& jobs) {
  int best = 0;
  double best_score = -1.0;
  for (int v = 0; v < 4; ++v) {
    long long tiles = 0;
    for (int j = 0; j < jobs.count; ++j) tiles += (jobs.job[j].M + kShapes[v].rows - 1) / kShapes[v].rows;
    const long long wg = tiles * ((N + kShapes[v].cols - 1) / kShapes[v].cols);
    const long long rounds = (wg + 255) / 256;
    const double score = (double)wg / (double)(rounds * 256) + 1e-3 * kShapes[v].rows * kShapes[v].cols / 4096.0;
    if (score > best_score) {
      best_score = score;
      best = v;
    }
  }
  return best;
}

template <typename T>
hipError_t near_launch(int n, int N, NearJobs jobs, const void* x, const void* gridbuf, const NearGrid& g,
                       hipStream_t s, int shape, int kind) {
  if (shape < 0 || shape >= kNumShapes) shape = near_default_shape(N, jobs);
  const NearShape sh = kShapes[shape];
  int tiles = 0;
  for (int j = 0; j < jobs.count; ++j) {
    jobs.job[j].tile0 = tiles;
    tiles += (jobs.job[j].M + sh.rows - 1) / sh.rows;
  }
  dim3 grid(tiles, (N + sh.cols - 1) / sh.cols);
  switch (shape) {
    case 0: launch_shape<T, 16, 256, 1, 8>(grid, s, kind, n, N, jobs, x, gridbuf, g); break;
    case 1: launch_shape<T, 32, 256, 1, 8>(grid, s, kind, n, N, jobs, x, gridbuf, g); break;
    case 2: launch_shape<T, 32, 128, 2, 8>(grid, s, kind, n, N, jobs, x, gridbuf, g); break;
    case 3: launch_shape<T, 64, 64, 4, 8>(grid, s, kind, n, N, jobs, x, gridbuf, g); break;
    case 4: launch_shape<T, 32, 64, 2, 8>(grid, s, kind, n, N, jobs, x, gridbuf, g); break;
    case 5: launch_shape<T, 16, 128, 1, 8>(grid, s, kind, n, N, jobs, x, gridbuf, g); break;
    case 6: launch_shape<T, 16, 64, 1, 8>(grid, s, kind, n, N, jobs, x, gridbuf, g); break;
    case 7: launch_shape<T, 32, 128, 2, 16>(grid, s, kind, n, N, jobs, x, gridbuf, g); break;
    case 8: launch_shape<T, 64, 64, 4, 16>(grid, s, kind, n, N, jobs, x, gridbuf, g); break;
    case 9: launch_shape<T, 16, 128, 1, 16>(grid, s, kind, n, N, jobs, x, gridbuf, g); break;
    default: launch_shape<T, 64, 128, 2, 8>(grid, s, kind, n, N, jobs, x, gridbuf, g); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t near_reduce_launch(const void* part, int ns, size_t len, void* y, void* y64, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<size_t>((len + 255) / 256, 8192);
  hipLaunchKernelGGL(near_reduce_kernel<T>, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const cplx<T>*>(part),
                     ns, len, reinterpret_cast<cplx<T>*>(y), reinterpret_cast<double2*>(y64));
  return hipGetLastError();
}

template hipError_t near_launch<double>(int, int, NearJobs, const void*, const void*, const NearGrid&, hipStream_t,
                                        int, int);
template hipError_t near_launch<float>(int, int, NearJobs, const void*, const void*, const NearGrid&, hipStream_t,
                                       int, int);
template hipError_t near_reduce_launch<double>(const void*, int, size_t, void*, void*, hipStream_t);
template hipError_t near_reduce_launch<float>(const void*, int, size_t, void*, void*, hipStream_t);

}  // namespace fmbem
