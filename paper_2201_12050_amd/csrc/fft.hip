// Multi-dimensional DFT over the (padded) cell grid, batched over channels.
//
// Layout [N3][N2][N1][channels] with channels contiguous, so every pass reads
// and writes whole channel rows (coalesced).  Forward transform with the sign
// of F_m = (e^{-2 pi i/m})^{jk} (Sec. 2.4); the inverse uses the conjugate
// kernel without the 1/m factor, which is folded into Lambda.  The pruned
// variants implement the incomplete Fourier matrices of Sec. 2.4: forward
// passes read only the first M_a inputs along each axis (the rest of the
// zero-padded input is never touched), inverse passes write only the first
// M_a outputs (the cropped rows are never computed).
//
// One workgroup handles one line of one axis for a tile of channels: the
// line is staged in LDS, twiddles come from a per-block LDS table, and each
// thread forms a set of outputs of one channel, eight at a time per sweep over
// the inputs.  Small grids of at most two transformed axes (N3 = 1) with few
// channels take a fused form instead: one workgroup per slice of channels does
// both axis passes through LDS in one launch (the separate passes are bound by
// launch and memory latency there, not by bandwidth).  Two more schedules use
// the matrix cores with the plan's DFT matrices: each axis pass as a GEMM
// (dft_gemm_launch), or both axes of an N3 = 1 grid in one launch with the
// slab of a 16-channel slice in LDS (dft2m_kernel, for many channels).
#include <algorithm>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "mfma.hpp"

namespace fmbem {

// channels per workgroup (16 complex doubles or 32 complex floats = 256 bytes per row),
// and output groups so that a workgroup has 256 threads
template <typename T> struct DftTile { static constexpr int ch = sizeof(T) == 8 ? 16 : 32; };
// built-in schedule (no measurement, e.g. engine rounds): the fused kernel up to this channel
// count (measured on a 32 x 32 grid: 121 channels 18.5 + 21.3 -> 14.6 + 14.1 us forward +
// inverse; from about 500 channels the separate passes are faster), above it the GEMM passes
// where they apply (faster than the direct passes from about 1000 channels), else the direct
// passes
constexpr int kDft2MaxChannels = 256;
// ... and the fused matrix-core kernel from this many channels (measured on the 8 x 8, 12 x 20 and
// 32 x 4 lattices: at 968 channels the GEMM passes are faster, at 7744 the fused kernel)
constexpr int kDftmMinChannels = 4096;

template <typename T>
__global__ __launch_bounds__(256) void dft_axis_kernel(cplx<T>* __restrict__ buf, int channels, int N, int Min,
                                                       int Mout, int sign, long long estride, int U,
                                                       long long su, long long sv, DftFlip flip) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* in = tw + N;  // [Min][kDftCh]
  constexpr int kDftCh = DftTile<T>::ch;
  constexpr int kDftGroups = 256 / kDftCh;
  const int tx = threadIdx.x % kDftCh;
  const int g = threadIdx.x / kDftCh;
  const int ch = blockIdx.x * kDftCh + tx;
  const int line = blockIdx.y;
  const int u = line % U, lv = line / U;
  cplx<T>* base = buf + u * su + lv * sv;
  for (int e = threadIdx.x; e < N; e += blockDim.x) {
    double s, c;
    sincospi(2.0 * e / N, &s, &c);
    tw[e] = mk<T>((T)c, (T)(sign * s));
  }
  const bool odd = flip.mode != 0 && ch < channels && odd_degree(ch, flip.p);
  for (int j = g; j < Min; j += kDftGroups) {
    cplx<T> v = ch < channels ? base[j * estride + ch] : mk<T>(0, 0);
    if (flip.mode == 2 && odd && bin_flipped(flip, j, u, lv)) v = mk<T>(-v.x, -v.y);
    in[j * kDftCh + tx] = v;
  }
  __syncthreads();
  if (ch >= channels) return;
  // each thread forms kOut outputs kk = g + kDftGroups (c kOut + q) of its channel per pass over
  // the inputs, reusing every staged input kOut times (twiddle reads are wave-uniform broadcasts)
  constexpr int kOut = 8;
  for (int c0 = g; c0 < Mout; c0 += kDftGroups * kOut) {
    cplx<T> acc[kOut];
    int e[kOut];
#pragma unroll
    for (int q = 0; q < kOut; ++q) {
      acc[q] = mk<T>(0, 0);
      e[q] = 0;
    }
    for (int j = 0; j < Min; ++j) {
      const cplx<T> x = in[j * kDftCh + tx];
#pragma unroll
      for (int q = 0; q < kOut; ++q) {
        const int kk = c0 + q * kDftGroups;
        if (kk < Mout) {
          cfma<T>(acc[q], x, tw[e[q]]);
          e[q] += kk;
          if (e[q] >= N) e[q] -= N;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kOut; ++q) {
      const int kk = c0 + q * kDftGroups;
      if (kk >= Mout) break;
      cplx<T> v = acc[q];
      if (flip.mode == 1 && odd && bin_flipped(flip, kk, u, lv)) v = mk<T>(-v.x, -v.y);
      base[kk * estride + ch] = v;
    }
  }
}

// Q outputs o = g + q G (q < Q, o < nout) of one line of a DFT: out[o] = sum_{j < nin} in[j stride]
// w^(j o), the twiddle index advanced by o per input (ascending j, as in dft_axis_kernel).
template <typename T, int Q>
__device__ inline void dft_line(const cplx<T>* in, size_t stride, int nin, const cplx<T>* tw, int N, int g, int G,
                                int nout, cplx<T> (&acc)[Q]) {
  int w[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    acc[q] = mk<T>(0, 0);
    w[q] = 0;
  }
#pragma unroll 8
  for (int j = 0; j < nin; ++j) {
    const cplx<T> x = in[(size_t)j * stride];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int o = g + q * G;
      if (o < nout) {
        cfma<T>(acc[q], x, tw[w[q]]);
        w[q] += o;
        if (w[q] >= N) w[q] -= N;
      }
    }
  }
}

// Fused two-axis DFT of a slice of CT channels (grid N0 x N1, N3 = 1), in place in the
// [N1][N0][channels] buffer.  Forward: the first M1 x M0 inputs -> axis 0 (M0 -> N0) ->
// axis 1 (M1 -> N1) -> all N1 x N0 bins, the symmetry factor D applied to the output.
// Inverse: all bins, D removed from the input -> axis 1 (N1 -> M1) -> axis 0 (N0 -> M0) ->
// the first M1 x M0 entries.  Every output is summed over its inputs in the order of
// dft_axis_kernel, so the result equals that of the two separate passes bit for bit.  Each
// thread forms kQ outputs of one line per sweep over its inputs (the loads of eight inputs in
// flight at once).
constexpr int kQ = 1;

__device__ inline bool flipped2(int k0, int k1, int N0, int N1) {
  const long long L = k0 + (long long)N0 * k1;
  const long long Lp = neg_mod(k0, N0) + (long long)N0 * neg_mod(k1, N1);
  return L > Lp;
}

template <typename T>
__global__ __launch_bounds__(256) void dft2_kernel(cplx<T>* __restrict__ buf, int channels, int CT, int N0, int N1,
                                                   int M0, int M1, int sign, int flip_p) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* tw0 = reinterpret_cast<cplx<T>*>(smem_raw);  // [N0]
  cplx<T>* tw1 = tw0 + N0;                              // [N1]
  cplx<T>* A = tw1 + N1;                                // staged inputs [rows][cols][CT]
  const bool inv = sign > 0;
  // forward: A = [M1][M0], Bm = [M1][N0] after axis 0; inverse: A = [N1][N0], Bm = [M1][N0] after axis 1
  cplx<T>* Bm = A + (size_t)(inv ? N1 * N0 : M1 * M0) * CT;
  const int c0 = blockIdx.x * CT;
  const int ct = min(CT, channels - c0);
  for (int e = threadIdx.x; e < N0; e += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * e / N0, &sn, &cs);
    tw0[e] = mk<T>((T)cs, (T)(sign * sn));
  }
  for (int e = threadIdx.x; e < N1; e += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * e / N1, &sn, &cs);
    tw1[e] = mk<T>((T)cs, (T)(sign * sn));
  }
  // stage the inputs of the slice (channel fastest)
  const int r_in = inv ? N1 : M1, c_in = inv ? N0 : M0;
  for (int e = threadIdx.x; e < r_in * c_in * ct; e += blockDim.x) {
    const int c = e % ct, t = e / ct;
    const int col = t % c_in, row = t / c_in;
    cplx<T> v = buf[((size_t)row * N0 + col) * channels + c0 + c];
    if (inv && flip_p > 0 && odd_degree(c0 + c, flip_p) && flipped2(col, row, N0, N1)) v = mk<T>(-v.x, -v.y);
    A[(size_t)t * CT + c] = v;
  }
  __syncthreads();
  cplx<T> acc[kQ];
  if (!inv) {
    // axis 0, lines i1 < M1: Bm[i1][k0] = sum_{i0 < M0} A[i1][i0] w0^(i0 k0)
    const int G0 = (N0 + kQ - 1) / kQ;
    for (int e = threadIdx.x; e < M1 * G0 * ct; e += blockDim.x) {
      const int c = e % ct, t = e / ct;
      const int g = t % G0, i1 = t / G0;
      dft_line<T, kQ>(A + (size_t)i1 * M0 * CT + c, CT, M0, tw0, N0, g, G0, N0, acc);
#pragma unroll
      for (int q = 0; q < kQ; ++q)
        if (g + q * G0 < N0) Bm[((size_t)i1 * N0 + g + q * G0) * CT + c] = acc[q];
    }
    __syncthreads();
    // axis 1, lines k0 < N0: out[k1][k0] = sum_{i1 < M1} Bm[i1][k0] w1^(i1 k1), D on the flipped bins
    const int G1 = (N1 + kQ - 1) / kQ;
    for (int e = threadIdx.x; e < N0 * G1 * ct; e += blockDim.x) {
      const int c = e % ct, t = e / ct;
      const int g = t % G1, k0 = t / G1;
      const bool odd = flip_p > 0 && odd_degree(c0 + c, flip_p);
      if (N1 > 1) {
        dft_line<T, kQ>(Bm + (size_t)k0 * CT + c, (size_t)N0 * CT, M1, tw1, N1, g, G1, N1, acc);
      } else {
        acc[0] = Bm[(size_t)k0 * CT + c];
      }
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int k1 = g + q * G1;
        if (k1 >= N1) break;
        cplx<T> v = acc[q];
        if (odd && flipped2(k0, k1, N0, N1)) v = mk<T>(-v.x, -v.y);
        buf[((size_t)k1 * N0 + k0) * channels + c0 + c] = v;
      }
    }
  } else {
    // axis 1, lines k0 < N0: Bm[i1][k0] = sum_{k1 < N1} A[k1][k0] w1^(k1 i1), i1 < M1
    const int G1 = (M1 + kQ - 1) / kQ;
    for (int e = threadIdx.x; e < N0 * G1 * ct; e += blockDim.x) {
      const int c = e % ct, t = e / ct;
      const int g = t % G1, k0 = t / G1;
      if (N1 > 1) {
        dft_line<T, kQ>(A + (size_t)k0 * CT + c, (size_t)N0 * CT, N1, tw1, N1, g, G1, M1, acc);
      } else {
        acc[0] = A[(size_t)k0 * CT + c];
      }
#pragma unroll
      for (int q = 0; q < kQ; ++q)
        if (g + q * G1 < M1) Bm[((size_t)(g + q * G1) * N0 + k0) * CT + c] = acc[q];
    }
    __syncthreads();
    // axis 0, lines i1 < M1: out[i1][i0] = sum_{k0 < N0} Bm[i1][k0] w0^(k0 i0), i0 < M0
    const int G0 = (M0 + kQ - 1) / kQ;
    for (int e = threadIdx.x; e < M1 * G0 * ct; e += blockDim.x) {
      const int c = e % ct, t = e / ct;
      const int g = t % G0, i1 = t / G0;
      dft_line<T, kQ>(Bm + (size_t)i1 * N0 * CT + c, CT, N0, tw0, N0, g, G0, M0, acc);
#pragma unroll
      for (int q = 0; q < kQ; ++q)
        if (g + q * G0 < M0) buf[((size_t)i1 * N0 + g + q * G0) * channels + c0 + c] = acc[q];
    }
  }
}

// Fused two-axis DFT on the matrix cores, for N3 = 1 grids with many channels and
// 1 < N_a <= kDftGemmMaxOut.  One workgroup of kDftmWaves waves per slice of kDftmCh channels (one
// tile column).  The slice's inputs are staged into LDS first with every load in flight at once (the
// D factor of the inverse removed on the way), then both axis passes run from LDS: each
// multiplies the lines of the slice by that axis's DFT matrix ([outputs][inputs]: forward
// [N_a][M_a], inverse [M_a][N_a]) on 16x16x4 tiles, a complex product as four real ones
// accumulated in the tile precision.  The first pass writes its outputs over its own inputs
// (a line only touches its own row or column of the slab), the second writes to the grid:
//   forward: X (M1 x M0) -> axis 0 -> T (M1 x N0) -> axis 1 -> all N1 x N0 bins, D applied;
//   inverse: all N1 x N0 bins -> axis 1 -> T (M1 x N0) -> axis 0 -> the first M1 x M0 entries.
// The slab has row stride N0: [M1][N0] forward, [N1][N0] inverse.
constexpr int kDftmCh = 16;
constexpr int kDftmGroup = 4;
#ifndef FMBEM_DFTM_WAVES
#define FMBEM_DFTM_WAVES 8
#endif
// waves per workgroup: two per SIMD, so that one wave's LDS reads overlap the other's MFMAs
constexpr int kDftmWaves = FMBEM_DFTM_WAVES;
constexpr int kDftmThreads = 64 * kDftmWaves;

// One sweep over the inputs of line L for output tiles mb0 .. mb0 + MBT - 1:
//   out(L, o, c) = sum_j A[o][j] in(L, j, c),  o in those tiles, o < nout.
// The k steps go four at a time, then the last one to three together (the matrix image is
// zero-padded to whole k steps and in() returns 0 past the last input): all fragments of a group
// are read first, then its MFMAs, with no branch inside a group, so the reads are issued together
// and the accumulators of consecutive MFMAs differ.
template <typename T, int MBT, typename In, typename Out>
__device__ inline void dftm_sweep(const cplx<T>* __restrict__ A, int lda, int mb0, int nout, int KS, int L, In in,
                                  Out out) {
  using MF = nmf<T>;
  using acc_t = typename MF::acc;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  acc_t re[MBT], im[MBT];
#pragma unroll
  for (int q = 0; q < MBT; ++q) {
    re[q] = acc_t{0, 0, 0, 0};
    im[q] = acc_t{0, 0, 0, 0};
  }
  const cplx<T>* Ar = A + (16 * mb0 + c) * lda + g;
  auto group = [&](int k0, auto nsteps) {
    constexpr int NS = decltype(nsteps)::value;
    cplx<T> x[NS], a[NS][MBT];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      x[u] = in(L, 4 * (k0 + u) + g, c);
#pragma unroll
      for (int q = 0; q < MBT; ++q) a[u][q] = Ar[16 * q * lda + 4 * (k0 + u)];
    }
#pragma unroll
    for (int u = 0; u < NS; ++u) {
#pragma unroll
      for (int q = 0; q < MBT; ++q) {
        re[q] = MF::step(a[u][q].x, x[u].x, re[q]);
        im[q] = MF::step(a[u][q].x, x[u].y, im[q]);
      }
#pragma unroll
      for (int q = 0; q < MBT; ++q) {
        re[q] = MF::step(-a[u][q].y, x[u].y, re[q]);
        im[q] = MF::step(a[u][q].y, x[u].x, im[q]);
      }
    }
  };
  int k0 = 0;
  for (; k0 + 4 <= KS; k0 += 4) group(k0, std::integral_constant<int, 4>{});
  // the last one to three k steps (wave-uniform)
  const int tail = KS - k0;
  if (tail == 3)
    group(k0, std::integral_constant<int, 3>{});
  else if (tail == 2)
    group(k0, std::integral_constant<int, 2>{});
  else if (tail == 1)
    group(k0, std::integral_constant<int, 1>{});
  // every input of the line has been read: the outputs may overwrite them
#pragma unroll
  for (int q = 0; q < MBT; ++q) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 16 * (mb0 + q) + MF::row(g, r);
      if (o < nout) out(L, o, c, mk<T>(re[q][r], im[q][r]));
    }
  }
}

// out(L, o, c) = sum_{j < nin} A[o][j] in(L, j, c) for o < nout and every line L = w + kDftmWaves i
// of wave w; the output tiles of a line in sweeps of at most kDftmGroup tiles.
template <typename T, typename In, typename Out>
__device__ inline void dftm_pass(const cplx<T>* __restrict__ A, int lda, int nout, int nin, int lines, In in,
                                 Out out) {
  // the wave index is uniform over the wave: made scalar so that the loops branch on scalars
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int MB = (nout + 15) >> 4, KS = (nin + 3) >> 2;
  for (int L = w; L < lines; L += kDftmWaves) {
    for (int mb0 = 0; mb0 < MB;) {
      const int rem = MB - mb0;
      if (rem >= 4) {
        dftm_sweep<T, 4>(A, lda, mb0, nout, KS, L, in, out);
        mb0 += 4;
      } else if (rem == 3) {
        dftm_sweep<T, 3>(A, lda, mb0, nout, KS, L, in, out);
        mb0 += 3;
      } else if (rem == 2) {
        dftm_sweep<T, 2>(A, lda, mb0, nout, KS, L, in, out);
        mb0 += 2;
      } else {
        dftm_sweep<T, 1>(A, lda, mb0, nout, KS, L, in, out);
        mb0 += 1;
      }
    }
  }
}

// padded LDS image of an [nout][nin] matrix: 16-row tiles, columns padded to whole k steps (4)
// plus one, the odd stride putting the 16 rows of a fragment in distinct banks
__host__ __device__ inline int dftm_rows(int nout) { return 16 * ((nout + 15) / 16); }
__host__ __device__ inline int dftm_lda(int nin) { return 4 * ((nin + 3) / 4) + 1; }

// FP32: at most 128 registers (two waves per SIMD); FP64 needs more for its register sets
template <typename T>
__global__ __launch_bounds__(kDftmThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 2 : 1))) void dft2m_kernel(
    cplx<T>* __restrict__ buf, int channels, int N0, int N1, int M0, int M1, int inverse, int flip_p,
    const cplx<T>* __restrict__ P1, const cplx<T>* __restrict__ P2) {
  extern __shared__ unsigned char smem_raw[];
  // pass 1 transforms axis 0 (forward) or axis 1 (inverse); pass 2 the other axis
  const int out1 = inverse ? M1 : N0, in1 = inverse ? N1 : M0;
  const int out2 = inverse ? M0 : N1, in2 = inverse ? N0 : M1;
  const int lda1 = dftm_lda(in1), lda2 = dftm_lda(in2);
  cplx<T>* A1 = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* A2 = A1 + (size_t)dftm_rows(out1) * lda1;
  cplx<T>* S = A2 + (size_t)dftm_rows(out2) * lda2;  // slab [rows][N0][kDftmCh]
  const int c0 = blockIdx.x * kDftmCh;
  const int c = threadIdx.x & 15;  // the channel of this thread in every staging step
  const int ch = c0 + c;
  const bool valid = ch < channels;
  const bool odd = valid && flip_p > 0 && odd_degree(ch, flip_p);
  auto sl = [&](int r, int k0, int cc) -> cplx<T>& { return S[((size_t)r * N0 + k0) * kDftmCh + cc]; };
  // stage the slab: forward X[i1][i0] (i1 < M1, i0 < M0); inverse Y[k1][k0], D removed.  With
  // 16-byte aligned channel rows (FP64 always, FP32 for an even channel count) every load takes
  // 16 bytes, two FP32 channels per thread; sixteen loads per thread are issued before their
  // LDS stores, so that enough bytes are in flight per CU to cover the memory latency.
  {
    const int rows = inverse ? N1 : M1, cols = inverse ? N0 : M0;
    constexpr int CPL = 16 / sizeof(cplx<T>);  // channels per 16-byte load
    if ((channels % CPL) == 0) {
      using V = typename Vec16<T>::type;
      constexpr int TPR = kDftmCh / CPL;       // threads per staged row of the slice
      const int cl = (threadIdx.x % TPR) * CPL;  // first channel of this thread in the slice
      const bool ok = c0 + cl < channels;        // whole load in range (channels % CPL == 0)
      bool odd2[CPL];
#pragma unroll
      for (int h = 0; h < CPL; ++h) odd2[h] = ok && flip_p > 0 && odd_degree(c0 + cl + h, flip_p);
      const int total = rows * cols * TPR;
#pragma unroll 16
      for (int e = threadIdx.x; e < total; e += kDftmThreads) {
        const int rc = e / TPR, col = rc % cols, row = rc / cols;
        V v{};
        if (ok) v = *reinterpret_cast<const V*>(buf + ((size_t)row * N0 + col) * channels + c0 + cl);
        cplx<T> u[CPL];
        memcpy(u, &v, sizeof(V));
        const bool fl = inverse && flipped2(col, row, N0, N1);
#pragma unroll
        for (int h = 0; h < CPL; ++h) {
          if (fl && odd2[h]) u[h] = mk<T>(-u[h].x, -u[h].y);
          sl(row, col, cl + h) = u[h];
        }
      }
    } else {
#pragma unroll 8
      for (int e = threadIdx.x; e < rows * cols * kDftmCh; e += kDftmThreads) {
        const int rc = e >> 4, col = rc % cols, row = rc / cols;
        cplx<T> v = valid ? buf[((size_t)row * N0 + col) * channels + ch] : mk<T>(0, 0);
        if (inverse && odd && flipped2(col, row, N0, N1)) v = mk<T>(-v.x, -v.y);
        sl(row, col, c) = v;
      }
    }
  }
#pragma unroll 4
  for (int e = threadIdx.x; e < dftm_rows(out1) * lda1; e += kDftmThreads) {
    const int r = e / lda1, k = e - r * lda1;
    A1[e] = (r < out1 && k < in1) ? P1[r * in1 + k] : mk<T>(0, 0);
  }
#pragma unroll 4
  for (int e = threadIdx.x; e < dftm_rows(out2) * lda2; e += kDftmThreads) {
    const int r = e / lda2, k = e - r * lda2;
    A2[e] = (r < out2 && k < in2) ? P2[r * in2 + k] : mk<T>(0, 0);
  }
  __syncthreads();
  if (!inverse) {
    // axis 0 over the rows i1 < M1, in place: T[i1][k0] = sum_{i0 < M0} F0[k0][i0] X[i1][i0]
    dftm_pass<T>(
        A1, lda1, N0, M0, M1, [&](int L, int j, int cc) { return j < M0 ? sl(L, j, cc) : mk<T>(0, 0); },
        [&](int L, int o, int cc, cplx<T> v) { sl(L, o, cc) = v; });
    __syncthreads();
    // axis 1 over the columns k0 < N0: Y[k1][k0] = sum_{i1 < M1} F1[k1][i1] T[i1][k0], D on flipped bins
    dftm_pass<T>(
        A2, lda2, N1, M1, N0, [&](int L, int j, int cc) { return j < M1 ? sl(j, L, cc) : mk<T>(0, 0); },
        [&](int L, int o, int, cplx<T> v) {
          if (!valid) return;
          if (odd && flipped2(L, o, N0, N1)) v = mk<T>(-v.x, -v.y);
          buf[((size_t)o * N0 + L) * channels + ch] = v;
        });
  } else {
    // axis 1 over the columns k0 < N0, in place: T[i1][k0] = sum_{k1 < N1} G1[i1][k1] Y[k1][k0]
    dftm_pass<T>(
        A1, lda1, M1, N1, N0, [&](int L, int j, int cc) { return j < N1 ? sl(j, L, cc) : mk<T>(0, 0); },
        [&](int L, int o, int cc, cplx<T> v) { sl(o, L, cc) = v; });
    __syncthreads();
    // axis 0 over the rows i1 < M1: X[i1][i0] = sum_{k0 < N0} G0[i0][k0] T[i1][k0], i0 < M0
    dftm_pass<T>(
        A2, lda2, M0, N0, M1, [&](int L, int j, int cc) { return j < N0 ? sl(L, j, cc) : mk<T>(0, 0); },
        [&](int L, int o, int, cplx<T> v) {
          if (valid) buf[((size_t)L * N0 + o) * channels + ch] = v;
        });
  }
}

template <typename T>
static size_t dftm_lds(const int M[3], const int N[3], bool inverse) {
  const int out1 = inverse ? M[1] : N[0], in1 = inverse ? N[1] : M[0];
  const int out2 = inverse ? M[0] : N[1], in2 = inverse ? N[0] : M[1];
  const size_t slab = (size_t)(inverse ? N[1] : M[1]) * N[0] * kDftmCh;
  return ((size_t)dftm_rows(out1) * dftm_lda(in1) + (size_t)dftm_rows(out2) * dftm_lda(in2) + slab) *
         sizeof(cplx<T>);
}

// LDS limit of one workgroup
constexpr size_t kLdsMax = 160 * 1024;

template <typename T>
bool dft_mfma_applies(int channels, const int M[3], const int N[3], bool pruned, const void* const* fmat) {
  if (!pruned || !fmat || channels < 1 || N[2] != 1 || M[2] != 1) return false;
  for (int a = 0; a < 2; ++a)
    if (N[a] <= 1 || N[a] > kDftGemmMaxOut || !fmat[a] || !fmat[3 + a]) return false;
  if ((long long)N[0] * N[1] * channels > INT32_MAX) return false;
  // the first pass works in place, so a line's outputs must come from one sweep over its inputs
  if (N[0] > 16 * kDftmGroup || M[1] > 16 * kDftmGroup) return false;
  return std::max(dftm_lds<T>(M, N, false), dftm_lds<T>(M, N, true)) <= kLdsMax;
}

// LDS budget of the fused form per workgroup
constexpr size_t kDft2Lds = 64 * 1024;

template <typename T>
static size_t dft2_per_channel(const int M[3], const int N[3], bool inverse) {
  return (size_t)(inverse ? N[1] * N[0] + M[1] * N[0] : M[1] * M[0] + M[1] * N[0]) * sizeof(cplx<T>);
}

template <typename T>
bool dft_fused_applies(int channels, const int M[3], const int N[3], bool pruned) {
  if (!pruned || N[2] != 1 || M[2] != 1 || N[0] <= 1 || channels < 1) return false;
  const size_t fixed = (size_t)(N[0] + N[1]) * sizeof(cplx<T>);
  const size_t per_ch = std::max(dft2_per_channel<T>(M, N, false), dft2_per_channel<T>(M, N, true));
  return fixed + per_ch <= kDft2Lds;
}

template <typename T>
bool dft_gemm_applies(int channels, const int M[3], const int N[3], bool pruned, const void* const* fmat) {
  if (!pruned || !fmat || channels < 1) return false;
  long long str = channels;
  for (int a = 0; a < 3; ++a) {
    if (N[a] > 1 && (!fmat[a] || !fmat[3 + a] || N[a] > kDftGemmMaxOut || str > INT32_MAX)) return false;
    str *= N[a];
  }
  return true;
}

// ---------------------------------------------------------------------------
// Schedule 4: both axes of an N3 = 1 grid in one launch as mixed-radix FFTs on the vector
// units.  A line of length N = P Q is split into P interleaved output sets: task t < P forms
// the outputs o = t + P s (s < Q) from the inputs j < nin as
//   z_t[q] = w^(q t) sum_u x[Q u + q] w^(Q u t)                (a pruned length-P stage, the "fold")
//   out[t + P s] = sum_{q < Q} z_t[q] e^(sign 2 pi i q s / Q)   (radix-2 length-Q DFT in registers)
// with w = e^(sign 2 pi i / N); this is exact because w^(j (t + P s)) = w^(j t) e^(sign 2 pi i (j mod Q) s / Q).
// A line costs about P nin + P Q (1 + log2 Q) complex operations against N nin for the direct
// DFT, only the inputs that exist are read (pruned input) and only the outputs that are kept are
// written (cropped output).  The radix Q of an axis depends on its length alone (the largest of
// 8, 4, 2, 1 dividing N), so every channel is summed in the same order whatever the number of
// channels.
//
// One workgroup per slice of CT channels; the slice's intermediate T (one transformed axis, the
// other still pruned) sits in LDS.  The axis transformed first is the one that makes the two
// passes cheaper (fewer fold products, see fft_first_axis).  Forward: pass A reads the inputs
// X (M1 x M0) from the grid and transforms axis a into T (M_b lines of N_a); pass B transforms
// axis b of T and writes all N1 x N0 bins (the factor D on the flipped bins of odd-degree
// channels).  Inverse: pass A reads all bins (D removed) and transforms axis a into T (N_b lines
// of M_a); pass B transforms axis b and writes the first M_b x M_a entries.  Every input of
// the slice is read in pass A and every output written in pass B, after a barrier, so the
// transform runs in place.  A task covers CP adjacent channels (one 16-byte access for two FP32
// or one FP64 channel), which share its twiddles.
template <typename T, int CP> struct FftPack { cplx<T> c[CP]; };

// a += b c as four fused multiply-adds (two per component)
__device__ inline void fcma(cplx<float>& a, cplx<float> b, cplx<float> c) {
  a.x = __builtin_fmaf(b.x, c.x, a.x);
  a.x = __builtin_fmaf(-b.y, c.y, a.x);
  a.y = __builtin_fmaf(b.x, c.y, a.y);
  a.y = __builtin_fmaf(b.y, c.x, a.y);
}
__device__ inline void fcma(cplx<double>& a, cplx<double> b, cplx<double> c) {
  a.x = __builtin_fma(b.x, c.x, a.x);
  a.x = __builtin_fma(-b.y, c.y, a.x);
  a.y = __builtin_fma(b.x, c.y, a.y);
  a.y = __builtin_fma(b.y, c.x, a.y);
}

// a b with an explicit rounding order (the same in every instantiation of the FFT kernels)
__device__ inline cplx<float> fcmul(cplx<float> a, cplx<float> b) {
  return mk<float>(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
__device__ inline cplx<double> fcmul(cplx<double> a, cplx<double> b) {
  return mk<double>(__builtin_fma(a.x, b.x, -(a.y * b.y)), __builtin_fma(a.x, b.y, a.y * b.x));
}

template <typename T, int CP>
__device__ inline FftPack<T, CP> fft_ld(const cplx<T>* p) {
  FftPack<T, CP> r;
  if constexpr (CP == 2) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    r.c[0] = mk<T>(v.x, v.y);
    r.c[1] = mk<T>(v.z, v.w);
  } else {
    r.c[0] = *p;
  }
  return r;
}

template <typename T, int CP>
__device__ inline void fft_st(cplx<T>* p, const FftPack<T, CP>& v) {
  if constexpr (CP == 2) {
    *reinterpret_cast<float4*>(p) = make_float4(v.c[0].x, v.c[0].y, v.c[1].x, v.c[1].y);
  } else {
    *p = v.c[0];
  }
}

// a * (S i), S = +1 or -1
template <int S, typename T>
__device__ inline cplx<T> mul_si(cplx<T> a) {
  return S > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

// in-place length-4 DFT with kernel e^(S 2 pi i / 4)
template <int S, typename T>
__device__ inline void dft4(cplx<T>& a0, cplx<T>& a1, cplx<T>& a2, cplx<T>& a3) {
  const cplx<T> s0 = cadd<T>(a0, a2), s1 = csub<T>(a0, a2), s2 = cadd<T>(a1, a3);
  const cplx<T> s3 = mul_si<S, T>(csub<T>(a1, a3));
  a0 = cadd<T>(s0, s2);
  a2 = csub<T>(s0, s2);
  a1 = cadd<T>(s1, s3);
  a3 = csub<T>(s1, s3);
}

// in-place length-Q DFT, out[s] = sum_q z[q] e^(S 2 pi i q s / Q), natural order (radix 2)
template <int Q, int S, typename T>
__device__ inline void dft_q(cplx<T> (&z)[Q]) {
  if constexpr (Q == 2) {
    const cplx<T> a = z[0], b = z[1];
    z[0] = cadd<T>(a, b);
    z[1] = csub<T>(a, b);
  } else if constexpr (Q == 4) {
    dft4<S, T>(z[0], z[1], z[2], z[3]);
  } else if constexpr (Q == 8) {
    cplx<T> e0 = z[0], e1 = z[2], e2 = z[4], e3 = z[6];
    cplx<T> o0 = z[1], o1 = z[3], o2 = z[5], o3 = z[7];
    dft4<S, T>(e0, e1, e2, e3);
    dft4<S, T>(o0, o1, o2, o3);
    // o_k *= e^(S 2 pi i k / 8): (1 + S i)/sqrt2, S i, (-1 + S i)/sqrt2
    const T h = (T)0.70710678118654752440;
    o1 = mk<T>(h * (o1.x - S * o1.y), h * (o1.y + S * o1.x));
    o2 = mul_si<S, T>(o2);
    o3 = mk<T>(h * (-o3.x - S * o3.y), h * (-o3.y + S * o3.x));
    z[0] = cadd<T>(e0, o0);
    z[4] = csub<T>(e0, o0);
    z[1] = cadd<T>(e1, o1);
    z[5] = csub<T>(e1, o1);
    z[2] = cadd<T>(e2, o2);
    z[6] = csub<T>(e2, o2);
    z[3] = cadd<T>(e3, o3);
    z[7] = csub<T>(e3, o3);
  }
}

// radix of an axis: the largest of 8, 4, 2 dividing its length, else 1 (a direct DFT)
__host__ __device__ inline int fft_radix(int N) { return N % 8 == 0 ? 8 : N % 4 == 0 ? 4 : N % 2 == 0 ? 2 : 1; }

// One pass over `lines` lines of length N = P Q: task (line L, residue t) of this thread's
// channel pack forms the outputs o = t + P s < nout of line L from its inputs j < nin.
// ld(L, j) returns a pack, st(L, o, pack) consumes one; tw[e] = e^(S 2 pi i e / N).  Tasks are
// dealt to the LS thread rows r0, r0 + LS, ... of the workgroup (the threads of one channel pack).
template <typename T, int CP, int Q, int S, typename Ld, typename St>
__device__ inline void fft_pass(int lines, int r0, int LS, int N, int nin, int nout, const cplx<T>* tw, Ld ld,
                                St st) {
  const int P = N / Q;
  const int tasks = lines * P;
  for (int id = r0; id < tasks; id += LS) {
    const int t = id % P, L = id / P;
    if (t >= nout) continue;  // every output of the task cropped (o = t + P s >= t)
    FftPack<T, CP> z[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int c = 0; c < CP; ++c) z[q].c[c] = mk<T>(0, 0);
    // fold: z[q] = sum_u x[Q u + q] w^(Q u t), the exponent Q u t kept below N
    const int step = Q * t;  // < N
    int e = 0;
    int j0 = 0;
    for (; j0 + Q <= nin; j0 += Q) {
      const cplx<T> w = tw[e];
      FftPack<T, CP> x[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) x[q] = ld(L, j0 + q);
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int c = 0; c < CP; ++c) fcma(z[q].c[c], x[q].c[c], w);
      e += step;
      if (e >= N) e -= N;
    }
    if (j0 < nin) {
      const cplx<T> w = tw[e];
#pragma unroll
      for (int q = 0; q < Q; ++q)
        if (j0 + q < nin) {
          const FftPack<T, CP> x = ld(L, j0 + q);
#pragma unroll
          for (int c = 0; c < CP; ++c) fcma(z[q].c[c], x.c[c], w);
        }
    }
    // z[q] *= w^(q t) (q t < N), then the length-Q DFT of every channel
#pragma unroll
    for (int q = 1; q < Q; ++q) {
      const cplx<T> w = tw[q * t];
#pragma unroll
      for (int c = 0; c < CP; ++c) z[q].c[c] = fcmul(z[q].c[c], w);
    }
#pragma unroll
    for (int c = 0; c < CP; ++c) {
      cplx<T> v[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) v[q] = z[q].c[c];
      dft_q<Q, S, T>(v);
#pragma unroll
      for (int q = 0; q < Q; ++q) z[q].c[c] = v[q];
    }
#pragma unroll
    for (int s = 0; s < Q; ++s) {
      const int o = t + P * s;
      if (o < nout) st(L, o, z[s]);
    }
  }
}

// the pass with the radix of its axis (runtime, uniform over the workgroup)
template <typename T, int CP, int S, typename Ld, typename St>
__device__ inline void fft_pass_q(int lines, int r0, int LS, int N, int nin, int nout, const cplx<T>* tw, Ld ld,
                                  St st) {
  switch (fft_radix(N)) {
    case 8: fft_pass<T, CP, 8, S>(lines, r0, LS, N, nin, nout, tw, ld, st); break;
    case 4: fft_pass<T, CP, 4, S>(lines, r0, LS, N, nin, nout, tw, ld, st); break;
    case 2: fft_pass<T, CP, 2, S>(lines, r0, LS, N, nin, nout, tw, ld, st); break;
    default: fft_pass<T, CP, 1, S>(lines, r0, LS, N, nin, nout, tw, ld, st); break;
  }
}

// whether bin (k0, k1) has a larger linear index k0 + N0 k1 than its partner (-k0, -k1)
__device__ inline bool bin_after_partner(int k0, int k1, int N0, int N1) {
  const int n1 = k1 == 0 ? 0 : N1 - k1;
  if (k1 != n1) return k1 > n1;
  return k0 > (k0 == 0 ? 0 : N0 - k0);
}

// fold products of the two passes (lines x residues x inputs) when axis a goes first
__host__ __device__ inline long long fft_cost(const int M[3], const int N[3], bool inverse, int a) {
  const int b = 1 - a;
  const long long Pa = N[a] / fft_radix(N[a]), Pb = N[b] / fft_radix(N[b]);
  if (!inverse) return (long long)M[b] * Pa * M[a] + (long long)N[a] * Pb * M[b];
  return (long long)N[b] * Pa * N[a] + (long long)M[a] * Pb * N[b];
}
__host__ __device__ inline int fft_first_axis(const int M[3], const int N[3], bool inverse) {
  return fft_cost(M, N, inverse, 1) < fft_cost(M, N, inverse, 0) ? 1 : 0;
}

// grid entry (k0, k1) at (k1 N0 + k0) channels; T entry (line, pos) at (line LT + pos) CT
template <typename T, int CP, int S>
__device__ inline void fft2_body(cplx<T>* __restrict__ buf, int channels, int CT, const int M[2], const int N[2],
                                 int a, int flip_p, const cplx<T>* twa, const cplx<T>* twb, cplx<T>* Tm, int blk) {
  const int b = 1 - a;
  const int c0 = blk * CT;
  const int NCP = CT / CP;
  const int npk = (min(CT, channels - c0) + CP - 1) / CP;  // packs of the slice in range
  // the block size is a multiple of NCP, so a thread keeps its channel pack in every task
  const int cp = threadIdx.x % NCP;
  const int r0 = threadIdx.x / NCP, LS = blockDim.x / NCP;
  const bool valid = cp < npk;
  int odd = 0;  // bit c: channel c of the pack has odd degree n (factor D of the spectrum symmetry)
  if (flip_p > 0 && valid)
#pragma unroll
    for (int c = 0; c < CP; ++c)
      if (odd_degree(c0 + cp * CP + c, flip_p)) odd |= 1 << c;
  auto negate = [&](FftPack<T, CP>& v) {
#pragma unroll
    for (int c = 0; c < CP; ++c)
      if (odd & (1 << c)) v.c[c] = mk<T>(-v.c[c].x, -v.c[c].y);
  };
  const long long sa = a == 0 ? channels : (long long)N[0] * channels;  // grid stride along axis a
  const long long sb = a == 0 ? (long long)N[0] * channels : channels;  // ... and along axis b
  cplx<T>* g = buf + c0 + cp * CP;
  cplx<T>* tp = Tm + cp * CP;
  // bin (ka, kb) -> (k0, k1)
  auto flipped = [&](int ka, int kb) {
    return a == 0 ? bin_after_partner(ka, kb, N[0], N[1]) : bin_after_partner(kb, ka, N[0], N[1]);
  };
  if (S < 0) {
    const int LT = N[a];  // T: M_b lines of N_a
    // pass A: lines kb < M_b, axis a (M_a inputs -> N_a outputs) into T
    if (valid)
      fft_pass_q<T, CP, S>(
          M[b], r0, LS, N[a], M[a], N[a], twa,
          [&](int L, int j) { return fft_ld<T, CP>(g + L * sb + j * sa); },
          [&](int L, int o, const FftPack<T, CP>& v) { fft_st<T, CP>(tp + ((size_t)L * LT + o) * CT, v); });
    __syncthreads();
    // pass B: lines ka < N_a, axis b (M_b inputs -> N_b outputs) to the grid, D on the flipped bins
    if (valid)
      fft_pass_q<T, CP, S>(
          N[a], r0, LS, N[b], M[b], N[b], twb,
          [&](int L, int j) { return fft_ld<T, CP>(tp + ((size_t)j * LT + L) * CT); },
          [&](int L, int o, FftPack<T, CP> v) {
            if (odd && flipped(L, o)) negate(v);
            fft_st<T, CP>(g + L * sa + o * sb, v);
          });
  } else {
    const int LT = M[a];  // T: N_b lines of M_a
    // pass A: lines kb < N_b, axis a (all N_a bins, D removed -> M_a outputs) into T
    if (valid)
      fft_pass_q<T, CP, S>(
          N[b], r0, LS, N[a], N[a], M[a], twa,
          [&](int L, int j) {
            FftPack<T, CP> v = fft_ld<T, CP>(g + L * sb + j * sa);
            if (odd && flipped(j, L)) negate(v);
            return v;
          },
          [&](int L, int o, const FftPack<T, CP>& v) { fft_st<T, CP>(tp + ((size_t)L * LT + o) * CT, v); });
    __syncthreads();
    // pass B: lines ia < M_a, axis b (N_b inputs -> the first M_b entries) to the grid
    if (valid)
      fft_pass_q<T, CP, S>(
          M[a], r0, LS, N[b], N[b], M[b], twb,
          [&](int L, int j) { return fft_ld<T, CP>(tp + ((size_t)j * LT + L) * CT); },
          [&](int L, int o, const FftPack<T, CP>& v) { fft_st<T, CP>(g + L * sa + o * sb, v); });
  }
}

constexpr int kFftThreads = 512;

// one plan's transform in a grouped launch: its grid, channel slices of CT channels, first axis,
// spectrum-symmetry flag and first workgroup
struct FftJob {
  void* buf;
  int channels, CT, N0, N1, M0, M1, a, flip_p, block0;
};
constexpr int kMaxFftJobs = 32;
struct FftJobs {
  int count;
  FftJob job[kMaxFftJobs];
};

// the transforms of several plans (same precision and channels per task) in one launch:
// workgroup blockIdx.x belongs to the last job whose block0 it reaches
template <typename T, int CP>
__global__ __launch_bounds__(kFftThreads) void fft2_kernel(FftJobs J, int inverse) {
  extern __shared__ unsigned char smem_raw[];
  int q = 0;
  while (q + 1 < J.count && (int)blockIdx.x >= J.job[q + 1].block0) ++q;
  const FftJob jb = J.job[q];
  const int N[2] = {jb.N0, jb.N1}, M[2] = {jb.M0, jb.M1};
  const int a = jb.a;
  cplx<T>* twa = reinterpret_cast<cplx<T>*>(smem_raw);  // [N_a]
  cplx<T>* twb = twa + N[a];                            // [N_b]
  constexpr int kAl = 16 / sizeof(cplx<T>);
  cplx<T>* Tm = twa + (N[0] + N[1] + kAl - 1) / kAl * kAl;  // the slab, 16-byte aligned
  const double sg = inverse ? 1.0 : -1.0;
  for (int e = threadIdx.x; e < N[0] + N[1]; e += blockDim.x) {
    const int n = e < N[a] ? N[a] : N[1 - a], k = e < N[a] ? e : e - N[a];
    double sn, cs;
    sincospi(2.0 * k / n, &sn, &cs);
    twa[e] = mk<T>((T)cs, (T)(sg * sn));
  }
  __syncthreads();
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(jb.buf);
  const int blk = (int)blockIdx.x - jb.block0;
  if (inverse)
    fft2_body<T, CP, 1>(buf, jb.channels, jb.CT, M, N, a, jb.flip_p, twa, twb, Tm, blk);
  else
    fft2_body<T, CP, -1>(buf, jb.channels, jb.CT, M, N, a, jb.flip_p, twa, twb, Tm, blk);
}

// LDS bytes of the FFT schedule for a slice of CT channels (the larger direction's slab)
template <typename T>
static size_t fft2_lds(const int M[3], const int N[3], int CT) {
  const size_t tw = (size_t)(N[0] + N[1] + 2) * sizeof(cplx<T>);
  size_t slab = 0;
  for (int inv = 0; inv < 2; ++inv) {
    const int a = fft_first_axis(M, N, inv != 0), b = 1 - a;
    slab = std::max(slab, (size_t)(inv ? N[b] * M[a] : M[b] * N[a]));
  }
  return tw + slab * CT * sizeof(cplx<T>);
}

template <typename T>
bool dft_fft_applies(int channels, const int M[3], const int N[3], bool pruned) {
  if (!pruned || channels < 1 || N[2] != 1 || M[2] != 1) return false;
  if ((long long)N[0] * N[1] * channels > INT32_MAX) return false;
  return fft2_lds<T>(M, N, 1) <= kLdsMax;
}

// channels per workgroup: 128 bytes of channels per grid entry (16 FP32 or 8 FP64), halved while
// the launch would have fewer than 64 workgroups (measured: more, narrower slices cost more in
// scattered writes than they gain in parallelism) or the slab would exceed 64 KB; CP channels per
// task (two FP32 channels in one 16-byte access when the channel count is even)
template <typename T>
static int fft2_cp(int channels) {
  return (sizeof(T) == 4 && channels % 2 == 0) ? 2 : 1;
}

template <typename T, int CP>
static hipError_t fft2_launch_jobs(const std::vector<FftTransform>& tr, bool inverse, hipStream_t s) {
  for (size_t i0 = 0; i0 < tr.size(); i0 += kMaxFftJobs) {
    FftJobs J{};
    size_t lds = 0;
    int threads = 64, blocks = 0;
    for (size_t i = i0; i < std::min(tr.size(), i0 + kMaxFftJobs); ++i) {
      const FftTransform& t = tr[i];
      int CT = 128 / (int)sizeof(cplx<T>);
      while (CT > CP && ((t.channels + CT - 1) / CT < 64 || fft2_lds<T>(t.M, t.N, CT) > 64 * 1024)) CT /= 2;
      const size_t l = fft2_lds<T>(t.M, t.N, CT);
      if (l > kLdsMax) return hipErrorInvalidValue;
      const int a = fft_first_axis(t.M, t.N, inverse), b = 1 - a;
      // threads: the larger pass's task count, whole waves, at most kFftThreads (any multiple of 64
      // is a multiple of the channel packs per slice, so that every thread keeps one pack)
      const int NCP = CT / CP;
      const int Pa = t.N[a] / fft_radix(t.N[a]), Pb = t.N[b] / fft_radix(t.N[b]);
      const long long ta = (long long)(inverse ? t.N[b] : t.M[b]) * Pa;
      const long long tb = (long long)(inverse ? t.M[a] : t.N[a]) * Pb;
      threads = (int)std::max<long long>(threads, std::min<long long>(kFftThreads, (std::max(ta, tb) * NCP + 63) / 64 * 64));
      lds = std::max(lds, l);
      FftJob& j = J.job[J.count++];
      j.buf = t.buf;
      j.channels = t.channels;
      j.CT = CT;
      j.N0 = t.N[0];
      j.N1 = t.N[1];
      j.M0 = t.M[0];
      j.M1 = t.M[1];
      j.a = a;
      j.flip_p = t.flip_p;
      j.block0 = blocks;
      blocks += (t.channels + CT - 1) / CT;
    }
    if (lds > 64 * 1024) {
      static std::once_flag once;
      static hipError_t attr = hipSuccess;
      std::call_once(once, [] {
        attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&fft2_kernel<T, CP>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
      });
      if (attr != hipSuccess) return attr;
    }
    hipLaunchKernelGGL((fft2_kernel<T, CP>), dim3(blocks), dim3(threads), lds, s, J, inverse ? 1 : 0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// the FFT schedule of several grids (every one an N3 = 1 grid where dft_fft_applies), in as few
// launches as their channels-per-task allow (one per precision and pairing of FP32 channels)
template <typename T>
hipError_t fft2_group_launch(const std::vector<FftTransform>& tr, bool inverse, hipStream_t s) {
  std::vector<FftTransform> one, two;
  for (const FftTransform& t : tr) (fft2_cp<T>(t.channels) == 2 ? two : one).push_back(t);
  hipError_t e = hipSuccess;
  if (!one.empty()) e = fft2_launch_jobs<T, 1>(one, inverse, s);
  if constexpr (sizeof(T) == 4)
    if (e == hipSuccess && !two.empty()) e = fft2_launch_jobs<T, 2>(two, inverse, s);
  return e;
}

template <typename T>
hipError_t grid_dft_launch(void* bufv, int channels, const int M[3], const int N[3], bool inverse, bool pruned,
                           hipStream_t s, int flip_p, int schedule, const void* const* fmat) {
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(bufv);
  if (schedule < 0) {
    if (dft_fft_applies<T>(channels, M, N, pruned))
      schedule = 4;
    else
      schedule = channels <= kDft2MaxChannels ? 1 : (channels >= kDftmMinChannels ? 3 : 2);
  }
  if (schedule == 4) {
    if (dft_fft_applies<T>(channels, M, N, pruned))
      return fft2_group_launch<T>({FftTransform{buf, channels, {M[0], M[1], M[2]}, {N[0], N[1], N[2]}, flip_p}},
                                  inverse, s);
    schedule = 0;
  }
  if (schedule == 3 && !dft_mfma_applies<T>(channels, M, N, pruned, fmat)) schedule = 2;
  if (schedule == 3) {
    const size_t lds = dftm_lds<T>(M, N, inverse);
    // dynamic LDS beyond 64 KB must be allowed per kernel
    static std::once_flag once;
    static hipError_t attr = hipSuccess;
    std::call_once(once, [] {
      attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&dft2m_kernel<T>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    });
    if (attr != hipSuccess) return attr;
    const int off = inverse ? 3 : 0;
    // pass 1 is axis 0 forward, axis 1 inverse
    const void* p1 = fmat[off + (inverse ? 1 : 0)];
    const void* p2 = fmat[off + (inverse ? 0 : 1)];
    hipLaunchKernelGGL(dft2m_kernel<T>, dim3((unsigned)((channels + kDftmCh - 1) / kDftmCh)), dim3(kDftmThreads), lds, s, buf,
                       channels, N[0], N[1], M[0], M[1], inverse ? 1 : 0, flip_p,
                       reinterpret_cast<const cplx<T>*>(p1), reinterpret_cast<const cplx<T>*>(p2));
    return hipGetLastError();
  }
  const bool gemm = schedule == 2 && dft_gemm_applies<T>(channels, M, N, pruned, fmat);
  if (schedule == 1 && dft_fused_applies<T>(channels, M, N, pruned)) {
    // channels per workgroup: enough workgroups to cover the CUs, within the LDS budget
    const size_t per_ch = dft2_per_channel<T>(M, N, inverse);
    const size_t fixed = (size_t)(N[0] + N[1]) * sizeof(cplx<T>);
    const int CT = std::max(1, std::min<int>((int)((kDft2Lds - fixed) / per_ch), (channels + 255) / 256));
    const int blocks = (channels + CT - 1) / CT;
    hipLaunchKernelGGL(dft2_kernel<T>, dim3(blocks), dim3(256), fixed + per_ch * CT, s, buf, channels, CT, N[0],
                       N[1], M[0], M[1], inverse ? 1 : -1, flip_p);
    return hipGetLastError();
  }
  long long str[3] = {channels, (long long)N[0] * channels, (long long)N[0] * N[1] * channels};
  int ext[3];
  for (int a = 0; a < 3; ++a) ext[a] = inverse ? N[a] : (pruned ? M[a] : N[a]);
  const int order_f[3] = {0, 1, 2}, order_i[3] = {2, 1, 0};
  // the pass that sees full bins: the last forward pass, the first inverse pass
  int edge = -1;
  for (int t = 0; t < 3; ++t) {
    const int a = inverse ? order_i[t] : order_f[t];
    if (N[a] > 1 && (inverse ? edge < 0 : true)) edge = a;
  }
  for (int t = 0; t < 3; ++t) {
    const int a = inverse ? order_i[t] : order_f[t];
    if (N[a] <= 1) continue;
    DftFlip fl{0, flip_p > 0 ? flip_p : 1, a, {N[0], N[1], N[2]}};
    if (flip_p > 0 && a == edge) fl.mode = inverse ? 2 : 1;
    const int b = (a == 0) ? 1 : 0;
    const int c = (a == 2) ? 1 : 2;
    const int Min = ext[a];
    const int Mout = inverse ? (pruned ? M[a] : N[a]) : N[a];
    const int lines = ext[b] * ext[c];
    if (gemm) {
      NearJob j{};
      j.A = buf;
      j.out = buf;
      j.src = fmat[(inverse ? 3 : 0) + a];
      j.M = channels;
      j.K = Min;
      j.N = Mout;
      j.lda = (int)str[a];
      j.batch = lines;
      j.src_kind = SRC_BATCH;
      j.dest = DEST_SLICE;
      hipError_t e = dft_gemm_launch<T>(j, DftGemm{str[b], str[c], ext[b], fl}, s);
      if (e != hipSuccess) return e;
      ext[a] = Mout;
      continue;
    }
    constexpr int ch = DftTile<T>::ch;
    dim3 grid((channels + ch - 1) / ch, lines);
    const size_t lds = (size_t)(N[a] + Min * ch) * sizeof(cplx<T>);
    hipLaunchKernelGGL(dft_axis_kernel<T>, grid, dim3(256), lds, s, buf, channels, N[a], Min, Mout,
                       inverse ? 1 : -1, str[a], ext[b], str[b], str[c], fl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ext[a] = Mout;
  }
  return hipSuccess;
}

template hipError_t grid_dft_launch<double>(void*, int, const int*, const int*, bool, bool, hipStream_t, int, int,
                                            const void* const*);
template hipError_t grid_dft_launch<float>(void*, int, const int*, const int*, bool, bool, hipStream_t, int, int,
                                           const void* const*);
template bool dft_gemm_applies<double>(int, const int*, const int*, bool, const void* const*);
template bool dft_gemm_applies<float>(int, const int*, const int*, bool, const void* const*);
template bool dft_fused_applies<double>(int, const int*, const int*, bool);
template bool dft_mfma_applies<double>(int, const int*, const int*, bool, const void* const*);
template bool dft_mfma_applies<float>(int, const int*, const int*, bool, const void* const*);
template bool dft_fused_applies<float>(int, const int*, const int*, bool);
template bool dft_fft_applies<double>(int, const int*, const int*, bool);
template bool dft_fft_applies<float>(int, const int*, const int*, bool);
template hipError_t fft2_group_launch<double>(const std::vector<FftTransform>&, bool, hipStream_t);
template hipError_t fft2_group_launch<float>(const std::vector<FftTransform>&, bool, hipStream_t);

}  // namespace fmbem
