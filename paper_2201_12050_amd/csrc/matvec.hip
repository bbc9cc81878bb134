// Operator application y = (S + U F^-1 Lambda F V) x  (Sec. 3.5, eq. (FMPBEMsystem)).
//
// Stream-ordered sequence on the caller's stream:
//   1. near field   y = sum_d S_d x_{c-d}                  (grouped GEMM, one segment per offset)
//   2. S2M          mhat[bin(c)][r] = V0 x_c               (GEMM into the padded grid)
//   3. forward DFT  over the cell grid, pruned inputs      (incomplete Fourier matrices, Sec. 2.4)
//   4. M2L          lhat_b = Lambda_b mhat_b               (per-bin product)
//   5. inverse DFT  cropped to the first M_a outputs per axis
//   6. L2T          y += U0 l_c                            (GEMM reading the padded grid)
#include <cmath>

#include "common.hpp"

namespace fmbem {

size_t matvec_workspace_bytes_per_rhs(const Plan& P, int precision) {
  const size_t el = precision == FMBEM_FP64 ? 16 : 8;
  const size_t b = (size_t)P.B * P.p * el;
  return (b + 255) / 256 * 256;
}

hipEvent_t prof_begin(const Plan& P, hipStream_t s) {
  if (!P.prof.on) return nullptr;
  hipEvent_t e = nullptr;
  if (!P.prof.pool.empty()) {
    e = P.prof.pool.back();
    P.prof.pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return nullptr;
  }
  hipEventRecord(e, s);
  return e;
}

void prof_end(const Plan& P, int stage, hipEvent_t start, hipStream_t s) {
  if (!start) return;
  hipEvent_t e = prof_begin(P, s);
  if (!e) return;
  P.prof.marks.push_back({stage, {start, e}});
}

template <typename T>
static hipError_t matvec_t(const Plan& P, int R, const void* x, void* y, void* ws, hipStream_t s) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const int n = P.n, C = P.C, p = P.p;
  const int N = R * C;
  hipEvent_t ev = prof_begin(P, s);
  // 1. near field
  {
    GemmSegs segs;
    segs.count = P.n_near;
    const size_t blk = (size_t)n * n * sizeof(cplx<T>);
    for (int d = 0; d < P.n_near; ++d) {
      segs.seg[d].A = reinterpret_cast<const char*>(P.S[prec]) + d * blk;
      segs.seg[d].d0 = P.near_off[3 * d];
      segs.seg[d].d1 = P.near_off[3 * d + 1];
      segs.seg[d].d2 = P.near_off[3 * d + 2];
    }
    GemmCols bm{COL_CELL_SHIFT, n, R, C, P.grid[0], P.grid[1], P.grid[2], P.fft[0], P.fft[1]};
    GemmCols cm{COL_LINEAR, n, R, C, P.grid[0], P.grid[1], P.grid[2], P.fft[0], P.fft[1]};
    hipError_t e = gemm_launch<T>(n, n, N, segs, x, bm, y, cm, false, s);
    if (e != hipSuccess) return e;
  }
  prof_end(P, 0 + 6 * prec, ev, s);
  if (P.n_far == 0) return hipSuccess;
  ev = prof_begin(P, s);
  // 2. S2M into the padded grid
  {
    GemmSegs segs;
    segs.count = 1;
    segs.seg[0] = GemmSeg{P.V0[prec], 0, 0, 0};
    GemmCols bm{COL_LINEAR, n, R, C, P.grid[0], P.grid[1], P.grid[2], P.fft[0], P.fft[1]};
    GemmCols cm{COL_CELL_TO_BIN, p, R, C, P.grid[0], P.grid[1], P.grid[2], P.fft[0], P.fft[1]};
    hipError_t e = gemm_launch<T>(p, n, N, segs, x, bm, ws, cm, false, s);
    if (e != hipSuccess) return e;
  }
  prof_end(P, 1 + 6 * prec, ev, s);
  // 3-5. DFT, M2L, inverse DFT
  ev = prof_begin(P, s);
  hipError_t e = grid_dft_launch<T>(ws, R * p, P.grid, P.fft, false, true, s);
  if (e != hipSuccess) return e;
  prof_end(P, 2 + 6 * prec, ev, s);
  ev = prof_begin(P, s);
  e = m2l_launch<T>(P.Lam[prec], ws, P.B, R, p, s);
  if (e != hipSuccess) return e;
  prof_end(P, 3 + 6 * prec, ev, s);
  ev = prof_begin(P, s);
  e = grid_dft_launch<T>(ws, R * p, P.grid, P.fft, true, true, s);
  if (e != hipSuccess) return e;
  prof_end(P, 4 + 6 * prec, ev, s);
  // 6. L2T accumulate
  ev = prof_begin(P, s);
  {
    GemmSegs segs;
    segs.count = 1;
    segs.seg[0] = GemmSeg{P.U0[prec], 0, 0, 0};
    GemmCols bm{COL_CELL_TO_BIN, p, R, C, P.grid[0], P.grid[1], P.grid[2], P.fft[0], P.fft[1]};
    GemmCols cm{COL_LINEAR, n, R, C, P.grid[0], P.grid[1], P.grid[2], P.fft[0], P.fft[1]};
    e = gemm_launch<T>(n, p, N, segs, ws, bm, y, cm, true, s);
  }
  prof_end(P, 5 + 6 * prec, ev, s);
  return e;
}

hipError_t matvec_launch(const Plan& P, int precision, int R, const void* x, void* y, void* ws, hipStream_t s) {
  return precision == FMBEM_FP64 ? matvec_t<double>(P, R, x, y, ws, s) : matvec_t<float>(P, R, x, y, ws, s);
}

}  // namespace fmbem

using namespace fmbem;

extern "C" fmbem_status fmbem_matvec(fmbem_plan plan, int32_t precision, int32_t n_rhs, const void* x, void* y,
                                     void* workspace, size_t workspace_bytes, void* hip_stream) {
  if (!plan || !x || !y || n_rhs < 1) return FMBEM_ERR_INVALID_ARG;
  if (precision != FMBEM_FP64 && precision != FMBEM_FP32) return FMBEM_ERR_INVALID_ARG;
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  if (!(P.precisions & (1u << precision))) return FMBEM_ERR_UNSUPPORTED;
  if ((size_t)n_rhs * P.C > (size_t)INT32_MAX / 2) return FMBEM_ERR_UNSUPPORTED;
  const size_t el = precision == FMBEM_FP64 ? 16 : 8;
  const size_t vbytes = (size_t)n_rhs * P.C * P.n * el;
  const char* xb = reinterpret_cast<const char*>(x);
  const char* yb = reinterpret_cast<const char*>(y);
  if (xb < yb + vbytes && yb < xb + vbytes) return FMBEM_ERR_INVALID_ARG;
  if (P.n_far > 0) {
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) return FMBEM_ERR_INVALID_ARG;
    if (workspace_bytes < (size_t)n_rhs * matvec_workspace_bytes_per_rhs(P, precision)) return FMBEM_ERR_WORKSPACE;
  }
  hipError_t e = matvec_launch(P, precision, n_rhs, x, y, workspace, reinterpret_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? FMBEM_OK : FMBEM_ERR_DEVICE;
}

extern "C" fmbem_status fmbem_plan_profile(fmbem_plan plan, int32_t enable) {
  if (!plan || (enable != 0 && enable != 1)) return FMBEM_ERR_INVALID_ARG;
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  if (enable) {
    for (auto& m : P.prof.marks) {
      hipEventSynchronize(m.second.second);
      P.prof.pool.push_back(m.second.first);
      P.prof.pool.push_back(m.second.second);
    }
    P.prof.marks.clear();
    for (int i = 0; i < FMBEM_N_STAGES; ++i) {
      P.prof.ms[i] = 0;
      P.prof.count[i] = 0;
    }
  }
  P.prof.on = enable != 0;
  return FMBEM_OK;
}

extern "C" fmbem_status fmbem_plan_profile_read(fmbem_plan plan, double* ms, int64_t* count) {
  if (!plan || !ms || !count) return FMBEM_ERR_INVALID_ARG;
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  for (auto& m : P.prof.marks) {
    float t = 0.f;
    if (hipEventSynchronize(m.second.second) != hipSuccess) return FMBEM_ERR_DEVICE;
    if (hipEventElapsedTime(&t, m.second.first, m.second.second) != hipSuccess) return FMBEM_ERR_DEVICE;
    P.prof.ms[m.first] += t;
    P.prof.count[m.first] += 1;
    P.prof.pool.push_back(m.second.first);
    P.prof.pool.push_back(m.second.second);
  }
  P.prof.marks.clear();
  for (int i = 0; i < FMBEM_N_STAGES; ++i) {
    ms[i] = P.prof.ms[i];
    count[i] = P.prof.count[i];
  }
  return FMBEM_OK;
}

extern "C" const char* fmbem_status_string(int32_t status) {
  switch (status) {
    case FMBEM_OK: return "ok";
    case FMBEM_ERR_INVALID_ARG: return "invalid argument";
    case FMBEM_ERR_UNSUPPORTED: return "unsupported";
    case FMBEM_ERR_OUT_OF_MEMORY: return "out of device memory";
    case FMBEM_ERR_DEVICE: return "device error";
    case FMBEM_ERR_NOT_CONVERGED: return "not converged";
    case FMBEM_ERR_WORKSPACE: return "workspace too small";
    default: return "unknown status";
  }
}
