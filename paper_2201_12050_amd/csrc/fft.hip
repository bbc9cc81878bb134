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
// launch and memory latency there, not by bandwidth).
#include <algorithm>

#include "common.hpp"

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

template <typename T>
hipError_t grid_dft_launch(void* bufv, int channels, const int M[3], const int N[3], bool inverse, bool pruned,
                           hipStream_t s, int flip_p, int schedule, const void* const* fmat) {
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(bufv);
  if (schedule < 0) schedule = channels <= kDft2MaxChannels ? 1 : 2;
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
template bool dft_fused_applies<float>(int, const int*, const int*, bool);

}  // namespace fmbem
