// Per-bin M2L product of the diagonalised far field (Sec. 2.4, eq. (diagonalized);
// Sec. 3.5, eq. (FMPBEMsystem)):  lhat_b = Lambda_b mhat_b  for every FFT bin b.
//
// Lambda_b (p x p, complex) is stored column-major per bin, so that the
// threads of a workgroup, one per output row, read consecutive addresses for
// every column j.  The product is in place in the [bin][R][p] spectrum buffer:
// each workgroup owns one bin, stages a group of up to kRhs right-hand-side
// vectors in LDS, and writes the results over them.
#include "common.hpp"

namespace fmbem {

constexpr int kRhs = 4;

template <typename T>
__global__ void m2l_gemv_kernel(const cplx<T>* __restrict__ Lam, cplx<T>* __restrict__ buf, int R, int p) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* xs = reinterpret_cast<cplx<T>*>(smem_raw);  // [kRhs][p]
  const int bin = blockIdx.x;
  const cplx<T>* Lb = Lam + (size_t)bin * p * p;
  cplx<T>* vb = buf + (size_t)bin * R * p;
  for (int r0 = 0; r0 < R; r0 += kRhs) {
    const int nr = min(kRhs, R - r0);
    __syncthreads();
    for (int t = threadIdx.x; t < nr * p; t += blockDim.x) xs[t] = vb[(size_t)r0 * p + t];
    __syncthreads();
    for (int i = threadIdx.x; i < p; i += blockDim.x) {
      cplx<T> acc[kRhs];
#pragma unroll
      for (int r = 0; r < kRhs; ++r) acc[r] = mk<T>(0, 0);
      for (int j = 0; j < p; ++j) {
        const cplx<T> a = Lb[(size_t)j * p + i];
#pragma unroll
        for (int r = 0; r < kRhs; ++r)
          if (r < nr) cfma<T>(acc[r], a, xs[r * p + j]);
      }
#pragma unroll
      for (int r = 0; r < kRhs; ++r)
        if (r < nr) vb[(size_t)(r0 + r) * p + i] = acc[r];
    }
  }
}

template <typename T>
hipError_t m2l_launch(const void* Lam, void* buf, int B, int R, int p, hipStream_t s) {
  const int threads = min(512, ((p + 63) / 64) * 64);
  hipLaunchKernelGGL(m2l_gemv_kernel<T>, dim3(B), dim3(threads), kRhs * p * sizeof(cplx<T>), s,
                     reinterpret_cast<const cplx<T>*>(Lam), reinterpret_cast<cplx<T>*>(buf), R, p);
  return hipGetLastError();
}

template hipError_t m2l_launch<double>(const void*, void*, int, int, int, hipStream_t);
template hipError_t m2l_launch<float>(const void*, void*, int, int, int, hipStream_t);

}  // namespace fmbem
