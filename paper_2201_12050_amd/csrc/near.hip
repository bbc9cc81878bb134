// Near field and S2M in one grouped launch (Sec. 3.2, eq. (2dPeriodicFMM); Sec. 3.5):
//
//   partial_d[:, (r,c)] = S_d x_{(r, c-d)}    for every near offset d   (n x n blocks)
//   mhat[bin(c)][r]     = V0 x_{(r, c)}                                  (p x n, into the padded grid)
//
// Every job is a complex GEMM with K = n (the unit-cell DOFs) whose B columns are
// the cells of x, shifted by the job's cell offset.  A workgroup owns a tile of
// kRows complex rows of one job and a chunk of kCols columns (cells x RHS), so
// the job's A tile is streamed from HBM once per column chunk while x stays in
// L2.  The per-offset partial products are summed afterwards in a fixed order
// (deterministic, independent of batching).  Complex arithmetic uses the
// real-split 2x2 form on 16x16x4 MFMA tiles (see gemm.hip); global loads for the
// next K step are issued before the MFMAs of the current one.
#include "common.hpp"

namespace fmbem {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

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

constexpr int kKc = 8;           // complex k per step

// Tile: ROWS complex rows x COLS columns, 4 waves arranged WR x (4/WR).
template <typename T, int ROWS, int COLS, int WR>
__global__ __launch_bounds__(256) void near_kernel(int n, int N, NearJobs jobs, const cplx<T>* __restrict__ x,
                                                   NearGrid g) {
  constexpr int WC = 4 / WR;
  constexpr int RR = 2 * ROWS;          // real rows per tile
  constexpr int RBW = RR / (16 * WR);   // 16-row MFMA blocks per wave
  constexpr int CBW = COLS / (16 * WC); // 16-column MFMA blocks per wave
  static_assert(RBW >= 1 && CBW >= 1, "tile too small for the wave grid");
  constexpr int LDA = RR + 4;
  constexpr int LDB = COLS + 4;
  constexpr int BPT = COLS * kKc / 256; // B complex elements per thread per step
  constexpr int TPC = kKc / BPT;        // threads per column
  __shared__ T As[2 * kKc][LDA];
  __shared__ T Bs[2 * kKc][LDB];
  using Acc = typename nmf<T>::acc;

  // job lookup
  int ji = 0;
  while (ji + 1 < jobs.count && (int)blockIdx.x >= jobs.job[ji + 1].tile0) ++ji;
  const NearJob jb = jobs.job[ji];
  const int m0 = ((int)blockIdx.x - jb.tile0) * ROWS;
  const int M = jb.M;
  const cplx<T>* A = reinterpret_cast<const cplx<T>*>(jb.A);
  const int col0 = blockIdx.y * COLS;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;

  // B column of this thread: cell shifted by the job offset, zero outside the grid
  const int b_col = tid / TPC;
  const int b_k = (tid % TPC) * BPT;
  const cplx<T>* bcol = nullptr;
  {
    const int j = col0 + b_col;
    if (j < N) {
      const int r = j / g.C;
      const int c = j - r * g.C;
      const int i1 = c % g.M0, t = c / g.M0;
      const int i2 = t % g.M1, i3 = t / g.M1;
      const int s1 = i1 - jb.d0, s2 = i2 - jb.d1, s3 = i3 - jb.d2;
      if (s1 >= 0 && s1 < g.M0 && s2 >= 0 && s2 < g.M1 && s3 >= 0 && s3 < g.M2)
        bcol = x + ((size_t)r * g.C + (s1 + g.M0 * (s2 + g.M1 * s3))) * n;
    }
  }
  // A staging: ROWS x kKc complex per step, APT per thread
  constexpr int AT = ROWS * kKc;
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
        const int m = m0 + e / kKc, kk = k0 + e % kKc;
        if (m < M && kk < n) ra[q] = A[(size_t)m * n + kk];
      }
    }
#pragma unroll
    for (int e = 0; e < BPT; ++e) rb[e] = mk<T>(0, 0);
    if (bcol) {
      if (k0 + kKc <= n) {
#pragma unroll
        for (int e = 0; e < BPT; ++e) rb[e] = bcol[k0 + b_k + e];
      } else {
        for (int e = 0; e < BPT; ++e)
          if (k0 + b_k + e < n) rb[e] = bcol[k0 + b_k + e];
      }
    }
  };
  load(0);
  for (int k0 = 0; k0 < n; k0 += kKc) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < APT; ++q) {
      const int e = tid + 256 * q;
      if (e < AT) {
        const int row = e / kKc, kc = e % kKc;
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
    if (k0 + kKc < n) load(k0 + kKc);
#pragma unroll
    for (int ks = 0; ks < 2 * kKc; ks += 4) {
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
#pragma unroll
  for (int j = 0; j < CBW; ++j) {
    const int col = col0 + 16 * (CBW * wc + j) + (lane & 15);
    if (col >= N) continue;
    cplx<T>* cc;
    if (jb.dest == 0) {
      cc = out + (size_t)col * M;
    } else {
      const int r = col / g.C;
      const int c = col - r * g.C;
      const int i1 = c % g.M0, t = c / g.M0;
      const int i2 = t % g.M1, i3 = t / g.M1;
      const size_t bin = (size_t)i1 + (size_t)g.N0 * (i2 + (size_t)g.N1 * i3);
      cc = out + (bin * g.R + r) * M;
    }
#pragma unroll
    for (int i = 0; i < RBW; ++i) {
      const int m = m0 + 8 * (RBW * wr + i) + 2 * (lane >> 4);
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (m + h < M) cc[m + h] = mk<T>(acc[i][j][2 * h], acc[i][j][2 * h + 1]);
    }
  }
}

// y[col][m] = sum_s part[s][col][m] in a fixed order
template <typename T>
__global__ void near_reduce_kernel(const cplx<T>* __restrict__ part, int ns, size_t len, cplx<T>* __restrict__ y) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (size_t)gridDim.x * blockDim.x) {
    cplx<T> s = part[i];
    for (int q = 1; q < ns; ++q) s = cadd<T>(s, part[(size_t)q * len + i]);
    y[i] = s;
  }
}

// tile shapes: (complex rows, columns, wave rows)
struct NearShape {
  int rows, cols, wr;
};
static const NearShape kShapes[] = {{16, 256, 1}, {32, 256, 1}, {32, 128, 2}, {64, 64, 4}, {32, 64, 2}, {16, 128, 1}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

int near_num_shapes() { return kNumShapes; }

template <typename T, int ROWS, int COLS, int WR>
static void launch_shape(dim3 grid, hipStream_t s, int n, int N, const NearJobs& jobs, const void* x,
                         const NearGrid& g) {
  hipLaunchKernelGGL((near_kernel<T, ROWS, COLS, WR>), grid, dim3(256), 0, s, n, N, jobs,
                     reinterpret_cast<const cplx<T>*>(x), g);
}

// default shape: the one whose workgroup count best fills whole rounds of 256 CUs
int near_default_shape(int N, const NearJobs& jobs) {
  int best = 0;
  double best_score = -1.0;
  for (int v = 0; v < kNumShapes; ++v) {
    long long tiles = 0;
    for (int j = 0; j < jobs.count; ++j) tiles += (jobs.job[j].M + kShapes[v].rows - 1) / kShapes[v].rows;
    const long long wg = tiles * ((N + kShapes[v].cols - 1) / kShapes[v].cols);
    const long long rounds = (wg + 255) / 256;
    // fill of the last round, and larger tiles (less L2 traffic per flop) on ties
    const double score = (double)wg / (double)(rounds * 256) + 1e-3 * kShapes[v].rows * kShapes[v].cols / 4096.0;
    if (v >= 4) continue;  // the small shapes are for the autotuner only
    if (score > best_score) {
      best_score = score;
      best = v;
    }
  }
  return best;
}

template <typename T>
hipError_t near_launch(int n, int N, NearJobs jobs, const void* x, const NearGrid& g, hipStream_t s, int shape) {
  if (shape < 0 || shape >= kNumShapes) shape = near_default_shape(N, jobs);
  const NearShape sh = kShapes[shape];
  int tiles = 0;
  for (int j = 0; j < jobs.count; ++j) {
    jobs.job[j].tile0 = tiles;
    tiles += (jobs.job[j].M + sh.rows - 1) / sh.rows;
  }
  dim3 grid(tiles, (N + sh.cols - 1) / sh.cols);
  switch (shape) {
    case 0: launch_shape<T, 16, 256, 1>(grid, s, n, N, jobs, x, g); break;
    case 1: launch_shape<T, 32, 256, 1>(grid, s, n, N, jobs, x, g); break;
    case 2: launch_shape<T, 32, 128, 2>(grid, s, n, N, jobs, x, g); break;
    case 3: launch_shape<T, 64, 64, 4>(grid, s, n, N, jobs, x, g); break;
    case 4: launch_shape<T, 32, 64, 2>(grid, s, n, N, jobs, x, g); break;
    default: launch_shape<T, 16, 128, 1>(grid, s, n, N, jobs, x, g); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t near_reduce_launch(const void* part, int ns, size_t len, void* y, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<size_t>((len + 255) / 256, 8192);
  hipLaunchKernelGGL(near_reduce_kernel<T>, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const cplx<T>*>(part),
                     ns, len, reinterpret_cast<cplx<T>*>(y));
  return hipGetLastError();
}

template hipError_t near_launch<double>(int, int, NearJobs, const void*, const NearGrid&, hipStream_t, int);
template hipError_t near_launch<float>(int, int, NearJobs, const void*, const NearGrid&, hipStream_t, int);
template hipError_t near_reduce_launch<double>(const void*, int, size_t, void*, hipStream_t);
template hipError_t near_reduce_launch<float>(const void*, int, size_t, void*, hipStream_t);

}  // namespace fmbem
