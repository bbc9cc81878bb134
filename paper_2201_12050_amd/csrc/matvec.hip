// Operator application y = (S + U F^-1 Lambda F V) x  (Sec. 3.5, eq. (FMPBEMsystem)).
//
// Stream-ordered sequence on the caller's stream (profiling stage in brackets):
//   [0] near field + S2M, one grouped launch:
//         part_d = S_d x_{c-d} for every near offset d, mhat[bin(c)][r] = V0 x_c
//   [2] forward DFT  over the cell grid, pruned inputs      (incomplete Fourier matrices, Sec. 2.4)
//   [3] M2L          lhat_b = Lambda_b mhat_b               (per-bin product)
//   [4] inverse DFT  cropped to the first M_a outputs per axis
//   [5] L2T          y = sum_d part_d + U0 l_c              (GEMM reading the padded grid, fixed-order sum)
//   [1] only without far-field offsets: y = sum_d part_d
//   [1] multilevel near field (FMPBEM2 plans, no dense near blocks): y += S~ x after [5]
// Workspace: [padded grid B x R x p][second grid][near partials n_near x R x C x n][multilevel
// buffers], 256-byte aligned.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "common.hpp"

namespace fmbem {

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

static size_t direct_ws_per_rhs(const Plan& P, int precision) {
  const size_t el = precision == FMBEM_FP64 ? 16 : 8;
  return 2 * align256((size_t)P.B * P.p * el) + align256((size_t)P.n_near * P.C * P.n * el) +
         ml_workspace_bytes_per_rhs(P, precision);
}

// workspace per RHS: the plan's own; with an image sub-plan (half-space periodic along z) also
// the input reversed along z, the image part's output and the sub-plan's workspace
size_t matvec_workspace_bytes_per_rhs(const Plan& P, int precision) {
  size_t b = direct_ws_per_rhs(P, precision);
  if (P.img) {
    const size_t el = precision == FMBEM_FP64 ? 16 : 8;
    b += 2 * align256((size_t)P.C * P.n * el) + direct_ws_per_rhs(*P.img, precision);
  }
  return b;
}

// a mark's time added to its stage (a mark carries the stage, with kProfUncounted for an interval
// that is not an application of its own)
static void prof_add(const Plan& P, int mark, float t) {
  const int stage = mark & ~kProfUncounted;
  if (stage < 0 || stage >= FMBEM_N_STAGES) return;
  P.prof.ms[stage] += t;
  if (!(mark & kProfUncounted)) P.prof.count[stage] += 1;
}

// completed marks: their times added to the stage totals, their events back in the pool
static void prof_harvest(const Plan& P) {
  size_t keep = 0;
  for (size_t i = 0; i < P.prof.marks.size(); ++i) {
    auto& m = P.prof.marks[i];
    float t = 0.f;
    if (hipEventQuery(m.second.second) == hipSuccess &&
        hipEventElapsedTime(&t, m.second.first, m.second.second) == hipSuccess) {
      prof_add(P, m.first, t);
      P.prof.pool.push_back(m.second.first);
      P.prof.pool.push_back(m.second.second);
    } else {
      P.prof.marks[keep++] = m;
    }
  }
  P.prof.marks.resize(keep);
}

// events come from the pool (filled when profiling starts and by completed marks), so that
// recording creates none while an application is timed
static hipEvent_t prof_record(const Plan& P, hipStream_t s) {
  hipEvent_t e = nullptr;
  if (P.prof.pool.empty()) prof_harvest(P);
  if (!P.prof.pool.empty()) {
    e = P.prof.pool.back();
    P.prof.pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return nullptr;
  }
  hipEventRecord(e, s);
  return e;
}

hipEvent_t prof_begin(const Plan& P, int stage, hipStream_t s) {
  if (!P.prof.active || !(P.prof.mask & (1u << stage))) return nullptr;
  return prof_record(P, s);
}

void prof_end(const Plan& P, int stage, hipEvent_t start, hipStream_t s, bool counted) {
  if (!start) return;
  hipEvent_t e = prof_record(P, s);
  if (!e) return;
  P.prof.marks.push_back({stage | (counted ? 0 : kProfUncounted), {start, e}});
}

// Autotuner of the tile shape of a grouped launch: on the first launch of a given
// job-list signature (kind, precision, job sizes), every shape is launched once to
// warm up and twice timed with HIP events on the caller's stream (the launches
// compute the real products, which the launch that follows overwrites); the fastest
// is cached for the process.  Blocks the host once per signature.
static std::mutex g_tune_mu;
static std::map<std::vector<long long>, int> g_tuned;

static bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

template <typename T>
int cached_shape(int kind, const std::vector<NearJob>& jobs);

template <typename T>
int tuned_shape(int kind, const std::vector<NearJob>& jobs, hipStream_t s) {
  // no timing launches into a stream that is being captured: a shape measured earlier or the default
  if (capturing(s)) return cached_shape<T>(kind, jobs);
  std::vector<long long> key{kind, (long long)sizeof(T)};
  for (const NearJob& j : jobs) {
    key.push_back(j.M);
    key.push_back(j.K);
    key.push_back(j.N);
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  int best = -1;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
    // two sweeps over the shapes, the minimum of each shape's timings counts
    const int ns = near_num_shapes<T>(kind);
    std::vector<float> t(ns, 1e30f);
    for (int sweep = 0; sweep < 2; ++sweep) {
      for (int v = 0; v < ns; ++v) {
        if (near_launch<T>(jobs, s, v, kind) != hipSuccess) continue;
        hipEventRecord(a, s);
        near_launch<T>(jobs, s, v, kind);
        near_launch<T>(jobs, s, v, kind);
        hipEventRecord(b, s);
        float ms = 0.f;
        if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) continue;
        t[v] = std::min(t[v], ms);
      }
    }
    for (int v = 0; v < ns; ++v)
      if (t[v] < 1e29f && (best < 0 || t[v] < t[best])) best = v;
    // the lowest-numbered shape within 2 % of the fastest: timing noise would otherwise flip the
    // choice between near-equal shapes from one process to the next
    if (best >= 0)
      for (int v = 0; v < best; ++v)
        if (t[v] <= 1.02f * t[best]) {
          best = v;
          break;
        }
  }
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = best;
  return best;
}

// tile shape of one of a plan's grouped launches (kind 0 near field + S2M, 1 L2T, 2 M2L GEMM):
// the plan's forced shape, else the tuned one (tune) or the cached / default one
template <typename T>
static int plan_shape(const Plan& P, int kind, const std::vector<NearJob>& jobs, hipStream_t s, bool tune) {
  if (P.tile_forced[kind] >= 0) return P.tile_forced[kind];
  return tune ? tuned_shape<T>(kind, jobs, s) : cached_shape<T>(kind, jobs);
}

// the tuned shape of this job-list signature if one was measured, else -1 (default shape)
template <typename T>
int cached_shape(int kind, const std::vector<NearJob>& jobs) {
  std::vector<long long> key{kind, (long long)sizeof(T)};
  for (const NearJob& j : jobs) {
    key.push_back(j.M);
    key.push_back(j.K);
    key.push_back(j.N);
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(key);
  return it == g_tuned.end() ? -1 : it->second;
}

// Autotuner of the DFT schedule (separate axis passes, the fused two-axis kernel, axis passes
// as MFMA GEMMs with the plan's DFT matrices, both axes fused on the matrix cores, or both axes
// as mixed-radix FFTs in one launch) of a plan's
// grid with R right-hand sides, chosen for the forward and the inverse transform separately: on
// the first application of a signature (precision, lattice, transform lengths, channels) where
// more than one schedule applies, each runs a forward and an inverse transform on the workspace
// grid (before the S2M product writes it) twice, timed with HIP events; the fastest of each
// direction is cached for the process.  Otherwise, or while the stream is being captured, a
// choice measured earlier or the built-in rule.  Returns forward | inverse << 4, or -1 for the
// built-in rule in both directions.
static inline int sched_fwd(int d) { return d < 0 ? -1 : (d & 15); }
static inline int sched_inv(int d) { return d < 0 ? -1 : (d >> 4); }

template <typename T>
static int dft_schedule(const Plan& P, int R, void* ws, hipStream_t s, bool tune) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const int ch = R * P.p;
  if (P.n_far == 0) return 0;
  constexpr int NS = 5;
  const bool ok[NS] = {true, dft_fused_applies<T>(ch, P.grid, P.fft, true),
                       dft_gemm_applies<T>(ch, P.grid, P.fft, true, P.dftF[prec]),
                       dft_mfma_applies<T>(ch, P.grid, P.fft, true, P.dftF[prec]),
                       dft_fft_applies<T>(ch, P.grid, P.fft, true)};
  if (!ok[1] && !ok[2] && !ok[3] && !ok[4]) return 0;
  if (P.dft_forced >= 0) {
    const int f = ok[P.dft_forced] ? P.dft_forced : 0;
    return f | (f << 4);
  }
  // where the FFT applies it is the fastest schedule (measured on the sphere lattices from 8 x 8 to
  // 32 x 32 at 1 to 64 right-hand sides) and it is not timed against the others: its result per
  // channel does not depend on the channel count, so an apply of many right-hand sides equals the
  // applies of each alone bit for bit
  if (ok[4]) return 4 | (4 << 4);
  const std::vector<long long> key{3, (long long)sizeof(T), P.grid[0], P.grid[1], P.grid[2],
                                   P.fft[0], P.fft[1], P.fft[2], ch};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  if (!tune || capturing(s)) return -1;
  hipEvent_t a = nullptr, b = nullptr, c = nullptr;
  float t[2][NS];
  for (int d = 0; d < 2; ++d)
    for (int v = 0; v < NS; ++v) t[d][v] = 1e30f;
  if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess && hipEventCreate(&c) == hipSuccess) {
    for (int sweep = 0; sweep < 2; ++sweep)
      for (int v = 0; v < NS; ++v) {
        if (!ok[v]) continue;
        if (grid_dft_launch<T>(ws, ch, P.grid, P.fft, false, true, s, P.flip_p(), v, P.dftF[prec]) != hipSuccess) continue;
        hipEventRecord(a, s);
        grid_dft_launch<T>(ws, ch, P.grid, P.fft, false, true, s, P.flip_p(), v, P.dftF[prec]);
        hipEventRecord(b, s);
        grid_dft_launch<T>(ws, ch, P.grid, P.fft, true, true, s, P.flip_p(), v, P.dftF[prec]);
        hipEventRecord(c, s);
        float ms0 = 0.f, ms1 = 0.f;
        if (hipEventSynchronize(c) != hipSuccess || hipEventElapsedTime(&ms0, a, b) != hipSuccess ||
            hipEventElapsedTime(&ms1, b, c) != hipSuccess)
          continue;
        t[0][v] = std::min(t[0][v], ms0);
        t[1][v] = std::min(t[1][v], ms1);
      }
  }
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  if (c) hipEventDestroy(c);
  int best[2] = {0, 0};
  for (int d = 0; d < 2; ++d)
    for (int v = 1; v < NS; ++v)
      if (t[d][v] < t[d][best[d]]) best[d] = v;
  const int code = best[0] | (best[1] << 4);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = code;
  return code;
}

// workspace layout: [padded grid B x R x p][second grid B x R x p][near partials n_near x R x C x n]
template <typename T>
static char* second_grid(const Plan& P, int R, void* ws) {
  return reinterpret_cast<char*>(ws) + align256((size_t)P.B * R * P.p * sizeof(cplx<T>));
}
template <typename T>
static char* near_partials(const Plan& P, int R, void* ws) {
  return reinterpret_cast<char*>(ws) + 2 * align256((size_t)P.B * R * P.p * sizeof(cplx<T>));
}
// buffers of the multilevel near field, after the near partials
template <typename T>
static char* ml_buffers(const Plan& P, int R, void* ws) {
  return near_partials<T>(P, R, ws) + align256((size_t)P.n_near * R * P.C * P.n * sizeof(cplx<T>));
}
// [1] the multilevel near field of an FMPBEM2 plan: y (+)= S~ x (after ml_s2m); parts as ml_apply.
// counted: the interval counts as one application of the stage (the other parts of a split
// application add their device time only)
template <typename T>
static hipError_t ml_stage(const Plan& P, int R, void* y, void* y64, void* ws, bool accum, hipStream_t s,
                           int parts = 15, bool counted = true) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  hipEvent_t ev = prof_begin(P, 1 + 6 * prec, s);
  const hipError_t e = ml_apply<T>(P, R, y, y64, ml_buffers<T>(P, R, ws), accum, s, parts);
  prof_end(P, 1 + 6 * prec, ev, s, counted);
  return e;
}
// [0] of an FMPBEM2 plan: the input in tree order and the S2M into the padded grid
template <typename T>
static hipError_t ml_s2m(const Plan& P, int R, const void* x, void* ws, hipStream_t s) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  hipEvent_t ev = prof_begin(P, 0 + 6 * prec, s);
  const hipError_t e = ml_prepare<T>(P, R, x, ml_buffers<T>(P, R, ws), ws, s);
  prof_end(P, 0 + 6 * prec, ev, s);
  return e;
}

// lhat_b = Lambda_b mhat_b for every bin: a GEMV in place for few right-hand sides, a
// batched MFMA GEMM into the second grid from kM2lGemmRhs on; returns the buffer of lhat
template <typename T>
static hipError_t m2l_apply(const Plan& P, int R, void* ws, hipStream_t s, void** lhat, bool tune) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  if (R < kM2lGemmRhs) {
    *lhat = ws;
    return m2l_launch<T>(P.Lam[prec], P.d_pairs, P.Bc, ws, R, P.p, s);
  }
  void* out = second_grid<T>(P, R, ws);
  NearJob j = near_job(P, R, P.Lam[prec], out, P.p, P.p, ws, SRC_BATCH, DEST_SLICE);
  j.N = R;
  j.lda = lambda_ld(P.p);
  j.batch = P.B;
  j.amap = P.d_canon;
  std::vector<NearJob> jobs{j};
  *lhat = out;
  return near_launch<T>(jobs, s, plan_shape<T>(P, 2, jobs, s, tune), 2);
}

template <typename T>
void near_s2m_jobs(const Plan& P, int R, const void* x, void* ws, std::vector<NearJob>& out) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const int n = P.n;
  const size_t el = sizeof(cplx<T>);
  char* part = near_partials<T>(P, R, ws);
  const size_t slice = (size_t)R * P.C * n;  // complex elements per near partial
  const size_t blk = (size_t)n * n * el;
  for (int d = 0; d < P.n_near; ++d) {
    NearJob j = near_job(P, R, reinterpret_cast<const char*>(P.S[prec]) + d * blk, part + d * slice * el, n, n, x,
                         SRC_X, DEST_SLICE);
    j.d0 = (short)P.near_off[3 * d];
    j.d1 = (short)P.near_off[3 * d + 1];
    j.d2 = (short)P.near_off[3 * d + 2];
    out.push_back(j);
  }
  // (FMPBEM2 plans: the S2M runs in ml_s2m)
  if (P.n_far > 0 && !P.ml) out.push_back(near_job(P, R, P.V0[prec], ws, P.p, n, x, SRC_X, DEST_GRID));
}

template <typename T>
NearJob l2t_job(const Plan& P, int R, void* ws, const void* lhat, void* y, void* y64) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  NearJob j = near_job(P, R, P.U0[prec], y, P.n, P.p, lhat, SRC_GRID, DEST_FINAL);
  j.part = near_partials<T>(P, R, ws);
  j.nparts = (short)P.n_near;
  j.out64 = y64;
  return j;
}

// Far-field chain of one plan on the plan's second stream, overlapping the near field on the
// caller's stream: fork after x is ready, S2M -> DFT -> M2L -> inverse DFT on the second
// stream, join before the L2T GEMM.  An FMPBEM2 plan gathers x into tree order before the fork,
// runs its S2M from it and, after the far chain, its exact leaf blocks on the second stream, and
// its tree stages (P2M up to the locals of the leaves) on the caller's stream; after the L2T it
// adds the L2P to the leaf-block output and that output to y.  Not used while the caller's stream
// is being captured.
template <typename T>
static hipError_t matvec_overlap(const Plan& P, int R, const void* x, void* y, void* ws, hipStream_t s, void* y64,
                                 bool tune) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const int n = P.n, p = P.p;
  const int dsched = dft_schedule<T>(P, R, ws, s, tune);
  std::lock_guard<std::mutex> lk(*P.aux_mu);
  hipError_t e;
  if (P.ml && (e = ml_prepare<T>(P, R, x, ml_buffers<T>(P, R, ws), ws, s, 1))) return e;
  if ((e = hipEventRecord(P.ev_fork, s))) return e;
  if ((e = hipStreamWaitEvent(P.aux, P.ev_fork, 0))) return e;
  // far chain [2]-[4] (S2M counted with the DFT stage)
  hipEvent_t ev = prof_begin(P, 2 + 6 * prec, P.aux);
  if (P.ml) {
    if ((e = ml_prepare<T>(P, R, x, ml_buffers<T>(P, R, ws), ws, P.aux, 2))) return e;
  } else {
    std::vector<NearJob> s2m{near_job(P, R, P.V0[prec], ws, p, n, x, SRC_X, DEST_GRID)};
    const int shape = plan_shape<T>(P, 0, s2m, P.aux, tune);
    if ((e = near_launch<T>(s2m, P.aux, shape, 0))) return e;
  }
  if ((e = grid_dft_launch<T>(ws, R * p, P.grid, P.fft, false, true, P.aux, P.flip_p(), sched_fwd(dsched), P.dftF[prec]))) return e;
  prof_end(P, 2 + 6 * prec, ev, P.aux);
  ev = prof_begin(P, 3 + 6 * prec, P.aux);
  void* lhat = nullptr;
  if ((e = m2l_apply<T>(P, R, ws, P.aux, &lhat, tune))) return e;
  prof_end(P, 3 + 6 * prec, ev, P.aux);
  ev = prof_begin(P, 4 + 6 * prec, P.aux);
  if ((e = grid_dft_launch<T>(lhat, R * p, P.grid, P.fft, true, true, P.aux, P.flip_p(), sched_inv(dsched), P.dftF[prec]))) return e;
  prof_end(P, 4 + 6 * prec, ev, P.aux);
  // the exact leaf blocks of an FMPBEM2 plan follow the far chain on the second stream
  if (P.ml && (e = ml_stage<T>(P, R, y, y64, ws, true, P.aux, 4, false))) return e;
  if ((e = hipEventRecord(P.ev_join, P.aux))) return e;
  // [0] near field on the caller's stream (the tree stages of an FMPBEM2 plan)
  if (P.ml) {
    if ((e = ml_stage<T>(P, R, y, y64, ws, true, s, 1))) return e;
  } else {
    std::vector<NearJob> jobs;
    near_s2m_jobs<T>(P, R, x, ws, jobs);
    jobs.pop_back();  // the S2M job ran on the second stream
    if (!jobs.empty()) {
      const int shape = plan_shape<T>(P, 0, jobs, s, tune);
      ev = prof_begin(P, 0 + 6 * prec, s);
      if ((e = near_launch<T>(jobs, s, shape, 0))) return e;
      prof_end(P, 0 + 6 * prec, ev, s);
    }
  }
  if ((e = hipStreamWaitEvent(s, P.ev_join, 0))) return e;
  // [5] L2T with the fixed-order sum of the near partials
  std::vector<NearJob> jobs{l2t_job<T>(P, R, ws, lhat, y, y64)};
  const int shape = plan_shape<T>(P, 1, jobs, s, tune);
  ev = prof_begin(P, 5 + 6 * prec, s);
  e = near_launch<T>(jobs, s, shape, 1);
  prof_end(P, 5 + 6 * prec, ev, s);
  if (e == hipSuccess && P.ml) e = ml_stage<T>(P, R, y, y64, ws, true, s, 8 | 2, false);
  return e;
}

template <typename T>
static hipError_t matvec_t(const Plan& P, int R, const void* x, void* y, void* ws, hipStream_t s, void* y64,
                           bool tune) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const int p = P.p;
  P.prof.active = P.prof.mask != 0 && (P.prof.calls++ % P.prof.period) == 0;
  // FP64, and FMPBEM2 plans: the FP32 near-field GEMM keeps every CU occupied until it drains, so a
  // concurrent far chain only delays it (measured on gfx950); the FP64 one leaves room, and so do
  // the short launches of the multilevel products
  if ((sizeof(T) == 8 || P.ml) && P.aux && P.n_far > 0 && !capturing(s))
    return matvec_overlap<T>(P, R, x, y, ws, s, y64, tune);
  const int dsched = dft_schedule<T>(P, R, ws, s, tune);
  // [0] near field and S2M
  hipEvent_t ev = nullptr;
  {
    std::vector<NearJob> jobs;
    near_s2m_jobs<T>(P, R, x, ws, jobs);
    if (!jobs.empty()) {
      const int shape = plan_shape<T>(P, 0, jobs, s, tune);
      ev = prof_begin(P, 0 + 6 * prec, s);
      hipError_t e = near_launch<T>(jobs, s, shape, 0);
      if (e != hipSuccess) return e;
    }
  }
  prof_end(P, 0 + 6 * prec, ev, s);
  if (P.ml) {
    hipError_t e = ml_s2m<T>(P, R, x, ws, s);
    if (e == hipSuccess && P.n_far == 0) e = ml_stage<T>(P, R, y, y64, ws, false, s);
    if (e != hipSuccess || P.n_far == 0) return e;
  }
  if (P.n_far == 0) {
    // [1] sum of the near partials
    ev = prof_begin(P, 1 + 6 * prec, s);
    hipError_t e = near_reduce_launch<T>(near_partials<T>(P, R, ws), P.n_near, (size_t)R * P.C * P.n, y, y64, s);
    if (e != hipSuccess) return e;
    prof_end(P, 1 + 6 * prec, ev, s);
    return hipSuccess;
  }
  // [2]-[4] DFT, M2L, inverse DFT
  ev = prof_begin(P, 2 + 6 * prec, s);
  hipError_t e = grid_dft_launch<T>(ws, R * p, P.grid, P.fft, false, true, s, P.flip_p(), sched_fwd(dsched), P.dftF[prec]);
  if (e != hipSuccess) return e;
  prof_end(P, 2 + 6 * prec, ev, s);
  ev = prof_begin(P, 3 + 6 * prec, s);
  void* lhat = nullptr;
  e = m2l_apply<T>(P, R, ws, s, &lhat, tune);
  if (e != hipSuccess) return e;
  prof_end(P, 3 + 6 * prec, ev, s);
  ev = prof_begin(P, 4 + 6 * prec, s);
  e = grid_dft_launch<T>(lhat, R * p, P.grid, P.fft, true, true, s, P.flip_p(), sched_inv(dsched), P.dftF[prec]);
  if (e != hipSuccess) return e;
  prof_end(P, 4 + 6 * prec, ev, s);
  // [5] L2T with the fixed-order sum of the near partials
  {
    std::vector<NearJob> jobs{l2t_job<T>(P, R, ws, lhat, y, y64)};
    const int shape = plan_shape<T>(P, 1, jobs, s, tune);
    ev = prof_begin(P, 5 + 6 * prec, s);
    e = near_launch<T>(jobs, s, shape, 1);
  }
  prof_end(P, 5 + 6 * prec, ev, s);
  if (e == hipSuccess && P.ml) e = ml_stage<T>(P, R, y, y64, ws, true, s);
  return e;
}

// Operator applications of several plans in one sequence, every stage in shared launches: the near
// field + S2M jobs of all of them in one grouped launch, then the forward grid FFTs of all of them,
// their GEMV M2L products and their M2L GEMMs, the inverse FFTs, and one grouped L2T launch (a plan
// whose DFT schedule is not the FFT, or whose M2L GEMM tile shape is forced, runs that stage in a
// launch of its own).  The grouped FFT and GEMV kernels sum every output of a plan in the same order
// as its own launch; the GEMM tile shapes are those tuned for the combined job list.  tune: autotune
// the tile shapes of the combined job lists (blocks the host once per composition); otherwise cached
// shapes or defaults.
template <typename T>
static hipError_t matvec_group_t(const std::vector<GroupApply>& g, hipStream_t s, bool tune) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  std::vector<NearJob> jobs;
  std::vector<int> dsched;
  for (const GroupApply& a : g) dsched.push_back(dft_schedule<T>(*a.P, a.R, a.ws, s, tune));
  for (const GroupApply& a : g) near_s2m_jobs<T>(*a.P, a.R, a.x, a.ws, jobs);
  int shape = -1;
  hipError_t e = hipSuccess;
  if (!jobs.empty()) {
    shape = tune ? tuned_shape<T>(0, jobs, s) : cached_shape<T>(0, jobs);
    if ((e = near_launch<T>(jobs, s, shape, 0)) != hipSuccess) return e;
  }
  std::vector<size_t> far;
  for (size_t q = 0; q < g.size(); ++q) {
    const GroupApply& a = g[q];
    const Plan& P = *a.P;
    if (P.ml && (e = ml_s2m<T>(P, a.R, a.x, a.ws, s)) != hipSuccess) return e;
    if (P.n_far == 0 && P.ml) {
      if ((e = ml_stage<T>(P, a.R, a.y, a.y64, a.ws, false, s)) != hipSuccess) return e;
    } else if (P.n_far == 0) {
      e = near_reduce_launch<T>(near_partials<T>(P, a.R, a.ws), P.n_near, (size_t)a.R * P.C * P.n, a.y, a.y64, s);
      if (e != hipSuccess) return e;
    } else {
      far.push_back(q);
    }
  }
  if (far.empty()) return hipSuccess;
  auto fft_ok = [&](size_t q, bool inv) {
    const GroupApply& a = g[q];
    const int sc = inv ? sched_inv(dsched[q]) : sched_fwd(dsched[q]);
    return sc == 4 && dft_fft_applies<T>(a.R * a.P->p, a.P->grid, a.P->fft, true);
  };
  // forward transforms
  std::vector<FftTransform> tr;
  for (size_t q : far) {
    const GroupApply& a = g[q];
    const Plan& P = *a.P;
    if (fft_ok(q, false)) {
      tr.push_back(FftTransform{a.ws, a.R * P.p, {P.grid[0], P.grid[1], P.grid[2]}, {P.fft[0], P.fft[1], P.fft[2]},
                                P.flip_p()});
    } else if ((e = grid_dft_launch<T>(a.ws, a.R * P.p, P.grid, P.fft, false, true, s, P.flip_p(), sched_fwd(dsched[q]),
                                       P.dftF[prec])) != hipSuccess) {
      return e;
    }
  }
  if (!tr.empty() && (e = fft2_group_launch<T>(tr, false, s)) != hipSuccess) return e;
  // per-bin M2L: GEMV products together, GEMMs together (into the second grid)
  std::vector<void*> lhat(g.size(), nullptr);
  std::vector<M2lProduct> gemv;
  std::vector<NearJob> gemm;
  for (size_t q : far) {
    const GroupApply& a = g[q];
    const Plan& P = *a.P;
    if (a.R < kM2lGemmRhs) {
      gemv.push_back(M2lProduct{P.Lam[prec], P.d_pairs, P.Bc, a.ws, a.R, P.p});
      lhat[q] = a.ws;
    } else if (P.tile_forced[2] >= 0) {
      if ((e = m2l_apply<T>(P, a.R, a.ws, s, &lhat[q], tune)) != hipSuccess) return e;
    } else {
      void* out = second_grid<T>(P, a.R, a.ws);
      NearJob j = near_job(P, a.R, P.Lam[prec], out, P.p, P.p, a.ws, SRC_BATCH, DEST_SLICE);
      j.N = a.R;
      j.lda = lambda_ld(P.p);
      j.batch = P.B;
      j.amap = P.d_canon;
      gemm.push_back(j);
      lhat[q] = out;
    }
  }
  if (!gemv.empty() && (e = m2l_group_launch<T>(gemv, s)) != hipSuccess) return e;
  if (!gemm.empty()) {
    shape = tune ? tuned_shape<T>(2, gemm, s) : cached_shape<T>(2, gemm);
    if ((e = near_launch<T>(gemm, s, shape, 2)) != hipSuccess) return e;
  }
  // inverse transforms
  tr.clear();
  for (size_t q : far) {
    const GroupApply& a = g[q];
    const Plan& P = *a.P;
    if (fft_ok(q, true)) {
      tr.push_back(FftTransform{lhat[q], a.R * P.p, {P.grid[0], P.grid[1], P.grid[2]},
                                {P.fft[0], P.fft[1], P.fft[2]}, P.flip_p()});
    } else if ((e = grid_dft_launch<T>(lhat[q], a.R * P.p, P.grid, P.fft, true, true, s, P.flip_p(),
                                       sched_inv(dsched[q]), P.dftF[prec])) != hipSuccess) {
      return e;
    }
  }
  if (!tr.empty() && (e = fft2_group_launch<T>(tr, true, s)) != hipSuccess) return e;
  std::vector<NearJob> l2t;
  for (size_t q : far) l2t.push_back(l2t_job<T>(*g[q].P, g[q].R, g[q].ws, lhat[q], g[q].y, g[q].y64));
  shape = tune ? tuned_shape<T>(1, l2t, s) : cached_shape<T>(1, l2t);
  if ((e = near_launch<T>(l2t, s, shape, 1)) != hipSuccess) return e;
  for (size_t q : far) {
    const GroupApply& a = g[q];
    if (a.P->ml && (e = ml_stage<T>(*a.P, a.R, a.y, a.y64, a.ws, true, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// xr[r][i0, i1, M2 - 1 - i2][:] = x[r][i0, i1, i2][:] (cells reversed along z)
template <typename T>
__global__ void reverse_z_kernel(const cplx<T>* __restrict__ x, cplx<T>* __restrict__ xr, int n, int M0, int M1,
                                 int M2, size_t total) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const size_t cellsz = (size_t)n;
  const size_t rc = idx / cellsz, i = idx - rc * cellsz;
  const int C = M0 * M1 * M2;
  const size_t r = rc / C;
  const int c = (int)(rc - r * C);
  const int i2 = c / (M0 * M1), rest = c - i2 * M0 * M1;
  const int cr = rest + M0 * M1 * (M2 - 1 - i2);
  xr[(r * C + cr) * cellsz + i] = x[idx];
}

// y += a (T), or y64 += a when y64 is set
template <typename T>
__global__ void add_kernel(cplx<T>* __restrict__ y, double2* __restrict__ y64, const cplx<T>* __restrict__ a,
                           size_t total) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const cplx<T> v = a[idx];
  if (y64) {
    y64[idx].x += (double)v.x;
    y64[idx].y += (double)v.y;
  } else {
    y[idx] = cadd<T>(y[idx], v);
  }
}

// the image part of a half-space plan periodic along z: y (or y64) += A_img (P x), the sub-plan
// applied to the input reversed along z; its buffers follow the plan's own workspace
template <typename T>
static hipError_t image_apply(const Plan& P, int R, const void* x, void* y, void* ws, hipStream_t s, void* y64,
                              bool tune) {
  const int prec = sizeof(T) == 8 ? FMBEM_FP64 : FMBEM_FP32;
  const size_t el = sizeof(cplx<T>);
  const size_t N = (size_t)P.C * P.n;
  char* base = reinterpret_cast<char*>(ws) + (size_t)R * direct_ws_per_rhs(P, prec);
  cplx<T>* xr = reinterpret_cast<cplx<T>*>(base);
  cplx<T>* yi = reinterpret_cast<cplx<T>*>(base + (size_t)R * align256(N * el));
  void* wsi = base + 2 * (size_t)R * align256(N * el);
  const size_t total = (size_t)R * N;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  hipLaunchKernelGGL(reverse_z_kernel<T>, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const cplx<T>*>(x), xr,
                     P.n, P.grid[0], P.grid[1], P.grid[2], total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = matvec_t<T>(*P.img, R, xr, yi, wsi, s, nullptr, tune)) != hipSuccess) return e;
  hipLaunchKernelGGL(add_kernel<T>, dim3(blocks), dim3(256), 0, s, reinterpret_cast<cplx<T>*>(y),
                     reinterpret_cast<double2*>(y64), yi, total);
  return hipGetLastError();
}

hipError_t matvec_group(int precision, const std::vector<GroupApply>& g, hipStream_t s, bool tune) {
  if (g.empty()) return hipSuccess;
  if (g.size() == 1)
    return matvec_launch(*g[0].P, precision, g[0].R, g[0].x, g[0].y, g[0].ws, s, g[0].y64, tune);
  hipError_t e = precision == FMBEM_FP64 ? matvec_group_t<double>(g, s, tune) : matvec_group_t<float>(g, s, tune);
  for (const GroupApply& a : g) {
    if (e != hipSuccess || !a.P->img) continue;
    e = precision == FMBEM_FP64 ? image_apply<double>(*a.P, a.R, a.x, a.y, a.ws, s, nullptr, tune)
                                : image_apply<float>(*a.P, a.R, a.x, a.y, a.ws, s, a.y64, tune);
  }
  return e;
}

hipError_t matvec_launch(const Plan& P, int precision, int R, const void* x, void* y, void* ws, hipStream_t s,
                         void* y64, bool tune) {
  hipError_t e = precision == FMBEM_FP64 ? matvec_t<double>(P, R, x, y, ws, s, nullptr, tune)
                                         : matvec_t<float>(P, R, x, y, ws, s, y64, tune);
  if (e != hipSuccess || !P.img) return e;
  return precision == FMBEM_FP64 ? image_apply<double>(P, R, x, y, ws, s, nullptr, tune)
                                 : image_apply<float>(P, R, x, y, ws, s, y64, tune);
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
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) return FMBEM_ERR_INVALID_ARG;
  if (workspace_bytes < (size_t)n_rhs * matvec_workspace_bytes_per_rhs(P, precision)) return FMBEM_ERR_WORKSPACE;
  hipError_t e = matvec_launch(P, precision, n_rhs, x, y, workspace, reinterpret_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? FMBEM_OK : FMBEM_ERR_DEVICE;
}

// ---------------------------------------------------------------------------
// Operator application without any allocation: the workspace is a static device array
// ---------------------------------------------------------------------------
// One array per device (each device that loads the library holds its own copy until the process
// ends).  Its device address is looked up once per device with hipGetSymbolAddress and kept; host
// code never passes the array's name itself (on the host it is only a stand-in symbol).
static __device__ __align__(256) unsigned char scratch[FMBEM_NOALLOC_WORKSPACE_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255)) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

extern "C" fmbem_status fmbem_matvec_noalloc(fmbem_plan plan, int32_t precision, int32_t n_rhs, const void* x,
                                             void* y, void* hip_stream) {
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
  if ((size_t)n_rhs * matvec_workspace_bytes_per_rhs(P, precision) > FMBEM_NOALLOC_WORKSPACE_BYTES)
    return FMBEM_ERR_WORKSPACE;
  void* ws = nullptr;
  if (scratch_address(P.device, &ws) != hipSuccess) return FMBEM_ERR_DEVICE;
  // no tile-shape or DFT-schedule timing (it would synchronise and create events): shapes measured
  // earlier for the same signature, else the defaults
  hipError_t e = matvec_launch(P, precision, n_rhs, x, y, ws, reinterpret_cast<hipStream_t>(hip_stream), nullptr,
                               false);
  return e == hipSuccess ? FMBEM_OK : FMBEM_ERR_DEVICE;
}

extern "C" fmbem_status fmbem_plan_profile(fmbem_plan plan, uint32_t stage_mask, int32_t period) {
  if (!plan || (stage_mask & ~FMBEM_PROFILE_ALL) || period < 1) return FMBEM_ERR_INVALID_ARG;
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  P.prof.period = period;
  P.prof.calls = 0;
  if (stage_mask) {
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
    while (P.prof.pool.size() < 256) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) break;
      P.prof.pool.push_back(e);
    }
  }
  P.prof.mask = stage_mask;
  return FMBEM_OK;
}

extern "C" fmbem_status fmbem_plan_profile_read(fmbem_plan plan, double* ms, int64_t* count) {
  if (!plan || !ms || !count) return FMBEM_ERR_INVALID_ARG;
  const Plan& P = *reinterpret_cast<Plan*>(plan);
  for (auto& m : P.prof.marks) {
    float t = 0.f;
    if (hipEventSynchronize(m.second.second) != hipSuccess) return FMBEM_ERR_DEVICE;
    if (hipEventElapsedTime(&t, m.second.first, m.second.second) != hipSuccess) return FMBEM_ERR_DEVICE;
    prof_add(P, m.first, t);
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
    case FMBEM_ERR_ADMISSION: return "request exceeds the engine's memory budget";
    default: return "unknown status";
  }
}
