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
// thread forms a set of outputs of one channel.
#include "common.hpp"

namespace fmbem {

// channels per workgroup (16 complex doubles or 32 complex floats = 256 bytes per row),
// and output groups so that a workgroup has 256 threads
template <typename T> struct DftTile { static constexpr int ch = sizeof(T) == 8 ? 16 : 32; };

template <typename T>
__global__ __launch_bounds__(256) void dft_axis_kernel(cplx<T>* __restrict__ buf, int channels, int N, int Min,
                                                       int Mout, int sign, long long estride, int U,
                                                       long long su, long long sv) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* in = tw + N;  // [Min][kDftCh]
  constexpr int kDftCh = DftTile<T>::ch;
  constexpr int kDftGroups = 256 / kDftCh;
  const int tx = threadIdx.x % kDftCh;
  const int g = threadIdx.x / kDftCh;
  const int ch = blockIdx.x * kDftCh + tx;
  const int line = blockIdx.y;
  const int u = line % U, v = line / U;
  cplx<T>* base = buf + u * su + v * sv;
  for (int e = threadIdx.x; e < N; e += blockDim.x) {
    double s, c;
    sincospi(2.0 * e / N, &s, &c);
    tw[e] = mk<T>((T)c, (T)(sign * s));
  }
  for (int j = g; j < Min; j += kDftGroups)
    in[j * kDftCh + tx] = ch < channels ? base[j * estride + ch] : mk<T>(0, 0);
  __syncthreads();
  if (ch >= channels) return;
  for (int kk = g; kk < Mout; kk += kDftGroups) {
    cplx<T> acc = mk<T>(0, 0);
    int e = 0;
    for (int j = 0; j < Min; ++j) {
      cfma<T>(acc, in[j * kDftCh + tx], tw[e]);
      e += kk;
      if (e >= N) e -= N * (e / N);
    }
    base[kk * estride + ch] = acc;
  }
}

template <typename T>
hipError_t grid_dft_launch(void* bufv, int channels, const int M[3], const int N[3], bool inverse, bool pruned,
                           hipStream_t s) {
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(bufv);
  long long str[3] = {channels, (long long)N[0] * channels, (long long)N[0] * N[1] * channels};
  int ext[3];
  for (int a = 0; a < 3; ++a) ext[a] = inverse ? N[a] : (pruned ? M[a] : N[a]);
  const int order_f[3] = {0, 1, 2}, order_i[3] = {2, 1, 0};
  for (int t = 0; t < 3; ++t) {
    const int a = inverse ? order_i[t] : order_f[t];
    if (N[a] <= 1) continue;
    const int b = (a == 0) ? 1 : 0;
    const int c = (a == 2) ? 1 : 2;
    const int Min = ext[a];
    const int Mout = inverse ? (pruned ? M[a] : N[a]) : N[a];
    const int lines = ext[b] * ext[c];
    constexpr int ch = DftTile<T>::ch;
    dim3 grid((channels + ch - 1) / ch, lines);
    const size_t lds = (size_t)(N[a] + Min * ch) * sizeof(cplx<T>);
    hipLaunchKernelGGL(dft_axis_kernel<T>, grid, dim3(256), lds, s, buf, channels, N[a], Min, Mout,
                       inverse ? 1 : -1, str[a], ext[b], str[b], str[c]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ext[a] = Mout;
  }
  return hipSuccess;
}

template hipError_t grid_dft_launch<double>(void*, int, const int*, const int*, bool, bool, hipStream_t);
template hipError_t grid_dft_launch<float>(void*, int, const int*, const int*, bool, bool, hipStream_t);

}  // namespace fmbem
