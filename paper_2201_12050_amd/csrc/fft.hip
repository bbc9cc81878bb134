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
// the inputs.
#include "common.hpp"

namespace fmbem {

// channels per workgroup (16 complex doubles or 32 complex floats = 256 bytes per row),
// and output groups so that a workgroup has 256 threads
template <typename T> struct DftTile { static constexpr int ch = sizeof(T) == 8 ? 16 : 32; };

// Spectrum symmetry: Lambda(-w) = D Lambda(w) D with D = diag((-1)^n) over the multipole
// index (n, m).  Bins whose linear index exceeds that of their partner -w carry the factor D
// (flip_mode 1: on the output of the last forward pass, 2: removed from the input of the
// first inverse pass), so that the M2L product can use the partner's Lambda.
struct DftFlip {
  int mode;       // 0 none, 1 output, 2 input
  int p;          // multipole coefficients per channel group
  int axis;       // transformed axis; the line index u, v runs over the other two (ascending)
  int N[3];       // full grid
};

__device__ inline bool bin_flipped(const DftFlip& f, int pos, int u, int v) {
  int c[3];
  const int b = f.axis == 0 ? 1 : 0, d = f.axis == 2 ? 1 : 2;
  c[f.axis] = pos;
  c[b] = u;
  c[d] = v;
  const long long L = c[0] + (long long)f.N[0] * (c[1] + (long long)f.N[1] * c[2]);
  const long long Lp = (f.N[0] - c[0]) % f.N[0] + (long long)f.N[0] * ((f.N[1] - c[1]) % f.N[1] +
                       (long long)f.N[1] * ((f.N[2] - c[2]) % f.N[2]));
  return L > Lp;
}

// (-1)^n of channel ch, whose multipole index is ch % p = n^2 + n + m
__device__ inline bool odd_degree(int ch, int p) {
  const int idx = ch % p;
  int n = (int)sqrtf((float)idx + 0.5f);
  while (n * n > idx) --n;
  while ((n + 1) * (n + 1) <= idx) ++n;
  return n & 1;
}

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

template <typename T>
hipError_t grid_dft_launch(void* bufv, int channels, const int M[3], const int N[3], bool inverse, bool pruned,
                           hipStream_t s, int flip_p) {
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(bufv);
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

template hipError_t grid_dft_launch<double>(void*, int, const int*, const int*, bool, bool, hipStream_t, int);
template hipError_t grid_dft_launch<float>(void*, int, const int*, const int*, bool, bool, hipStream_t, int);

}  // namespace fmbem
