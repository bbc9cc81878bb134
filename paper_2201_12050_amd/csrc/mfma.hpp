// 16x16x4 matrix-core tiles (gfx950) shared by the GEMM, DFT and multilevel product kernels.
#pragma once

#include "common.hpp"

namespace fmbem {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; };
template <> struct Vec16<double> { using type = double2; };

// Output layout of the 16x16x4 tiles (checked on gfx950): lane l holds column l % 16
// and four rows q = 0..3: f32 rows 4g + q, f64 rows g + 4q (g = l / 16).
template <typename T> struct nmf;
template <> struct nmf<double> {
  using acc = v4d;
  __device__ static inline int row(int g, int q) { return g + 4 * q; }
  __device__ static inline acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct nmf<float> {
  using acc = v4f;
  __device__ static inline int row(int g, int q) { return 4 * g + q; }
  __device__ static inline acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

}  // namespace fmbem
