// Multilevel near field of FMPBEM2 (Sec. 3.3): every near block S_d applied as a
// multilevel FMM over the boxes of the lattice instead of as a dense n x n block.
//
// Subdivision: the lattice box of the unit cell (edge = pitch per axis, centred on the cell
// centre) is halved L times along every axis; an element belongs to the box holding its
// centroid.  The boxes of one level of the whole lattice lie on one regular grid (edge
// h_l = pitch / 2^l), and two boxes are well separated when their grid offset has Chebyshev
// norm >= 2 (eq. (admissibility) with r the box edge; on level 0, the cells, that is the far
// set of the single-level FMPBEM).  Descending from the pairs (cell i, cell i - d) of the
// near offsets d, a pair of boxes is translated by M2L on the first level on which it is well
// separated; pairs of leaves that are near on every level take the exact entries of S_d
// (P2P).  Moments: P2M about the leaf centres (eq. (p2m)), M2M up to level 1 (eq. (m2m));
// locals: M2L (eq. (m2l)), L2L down to the leaves (eq. (l2l)), L2P (eq. (l2p)); truncation
// n_t,near.  Every cell has the same tree, so each interaction list is one list of (target
// box, source box, cell offset) entries applied to every cell of the lattice at once.
//
// Translation matrices (host, FP64): with G(a,alpha; b,beta; c,gamma) = (a b c;0 0 0)
// (a b c;alpha beta gamma), evaluated as the Gaunt integral 1/2 int Yt_a^alpha Yt_b^beta
// Yt_c^gamma dx,
//   M2M (b = y_c - y_c'):  T[(n,m),(n',m')] = (2n'+1)(-1)^{m'} sum_l (2l+1) i^{n'-n+l}
//                                             G(n',-m'; n,m; l,m'-m) I_l^{m'-m}(b)
//   L2L (b = x_c' - x_c):  T[(n,m),(n',m')] = (2n'+1)(-1)^m sum_l (2l+1) i^{n-n'+l}
//                                             G(n,-m; n',m'; l,m-m') I_l^{m-m'}(b)
//   M2L: the cell-level table of plan.hip with O_l^mu at the box-centre offset.
// Each level carries the diagonal scaling s_l^n (s_l = k times the box half-diagonal,
// clamped to [1e-3, 1]): moments / s_l^n, locals * s_l^n, so that FP32 stays in range.
//
// Application (all cells and right-hand sides at once): the input is gathered into tree
// order with the columns (RHS r, cell c) innermost, then every stage is one launch of the
// block-sparse product kernel -- the P2P blocks (from the input alone, so they may run beside
// the tree stages), P2M, M2M per level, M2L of all levels, L2L per level, and the L2P added to
// the P2P output -- and the result is scattered back and added to y.  Targets of more than 32
// expansion rows are split into row blocks, and the two heavy stages (M2L, P2P) divide each
// target's tasks over several workgroups whose partial sums are added in slot order afterwards.
// The S2M of the cell-level far field reads the same tree-ordered input as a split-K product
// (partial sums over element chunks, added in chunk order).  Every sum runs in a fixed order,
// so an application's result does not depend on timing.
#include <algorithm>
#include <array>
#include <cmath>
#include <functional>
#include <map>
#include <numeric>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "mfma.hpp"
#include "specfun.hpp"

namespace fmbem {

constexpr int kMlRows = 64;  // rows of one S2M output block (the largest target of any stage)
constexpr int kMlZeroShift = 13;
constexpr int kMlS2mChunk = 128;  // elements per partial sum of the S2M
constexpr int kMlLeafRows = 32;   // element rows of one L2P / P2P output block

// ---------------------------------------------------------------------------
// device: block-sparse products
// ---------------------------------------------------------------------------
struct MlBufs {
  void* b[7];  // 0: input in tree order, 1: moments, 2: locals, 3: output in tree order ([row][cols]),
               // 4: S2M partial sums, 5: partial sums of the split M2L, 6: of the split P2P stage
};

// a complex zero in device memory (never written), read in place of entries outside the operands
__device__ double2 ml_zero_entry;

// *p when c, else 0: one unconditional load from p or from the zero entry (a guarded load, or a
// select after the load, makes the wave wait for the data at once instead of at its use)
template <typename T>
__device__ inline cplx<T> load_if(const cplx<T>* p, bool c) {
  return *(c ? p : reinterpret_cast<const cplx<T>*>(&ml_zero_entry));
}

// the waves of one stream agree on its LDS staging area: a workgroup barrier when a stream spans
// several waves; a single wave's LDS operations complete in issue order, so it only needs the
// compiler to keep them in program order
// sum over the 64 lanes of a wave (every lane gets it)
__device__ inline int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int SLICES>
__device__ inline void stream_sync() {
  if constexpr (SLICES == 1) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// out[out_row + i][col] (+)= sum over the target's tasks of A[i][k] src[src_row + k][col'] with
// col' the column of cell c - d (zero outside the lattice), on the 16x16x4 matrix cores.  The
// target's work is a list of items (task, KW-wide contraction chunk).  The workgroup's 4 waves
// form WS streams of 4 / WS column slices of 16, stream j taking items j, j + WS, ...  Every round
// each stream stages its item (A chunk ROWS x KW and source chunk KW x its columns, zero beyond
// the target's rows, the item's contraction and the lattice) in its own LDS region while the
// next item is loaded into registers; each wave then multiplies its RT row tiles of 16 by its
// column slice with four real products per complex product and k step of 4.  The streams'
// partial sums are added in stream order.  Occupancy: 4 waves per SIMD for up to 32 rows.
// Measured on the 4 x 4 lattice of 20480-triangle cells (4 levels, n_t,near = 4; whole multilevel
// near field, FP32 / FP64), step by step from the first form of this loop: the matrix cores in
// place of the vector ALU (one lane per column, RT rows per lane, nine complex LDS operands per
// eight multiply-adds) 334 -> 288 us / 429 -> 389 us; no workgroup barrier per round where a
// stream is a single wave -> 246 / 360; the task descriptors in lanes instead of a dependent load
// per task -> 244 / 326; 4 waves per SIMD -> 221 / 285; unconditional loads (a guarded load, or a
// select right after the load, waited for the operands at once) -> 183 / 274.  A second item in
// flight (two register sets) was 5-10 % slower; FP32 chunks of 8 were 3 % slower and of 32 (fewer
// waves per SIMD) 23 % slower than 16.
template <typename T, int WS, int RT, int KW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RT <= 2 ? 4 : 1))) void ml_kernel(
    const MlTarget* __restrict__ tg, const MlTask* __restrict__ tk, const cplx<T>* __restrict__ ops, MlBufs B,
    int out_id, int accum, int cols, int C, int M0, int M1, int M2) {
  static_assert(KW % 4 == 0, "whole k steps");
  using mf = nmf<T>;
  using acc_t = typename mf::acc;
  constexpr int SLICES = 4 / WS, ROWS = 16 * RT;
  constexpr int SC = SLICES * 16;               // columns of a stream
  constexpr int STG = (ROWS * KW + SLICES * 64 - 1) / (SLICES * 64);  // A entries staged per thread and item
  constexpr int XSTG = KW * SC / (SLICES * 64);   // source entries staged per thread and item
  __shared__ cplx<T> As[WS][KW][ROWS + 1];
  __shared__ cplx<T> Xs[WS][KW][SC];
  // the streams' reduction area: the staging area when it is large enough
  constexpr bool kAlias = ROWS * SC <= WS * KW * (ROWS + 1);
  __shared__ cplx<T> red_own[(WS > 1 && !kAlias) ? ROWS * SC : 1];
  cplx<T>* red = kAlias ? &As[0][0][0] : red_own;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int stream = wave / SLICES, slice = wave - stream * SLICES;
  const int ts = slice * 64 + lane;  // thread index within the stream
  const int li = lane & 15, g = lane >> 4;
  const MlTarget t = tg[blockIdx.x];
  const int col0 = blockIdx.y * SC;
  // the column this thread loads (the same for every entry it stages, since SC divides SLICES 64)
  const int lcol = col0 + ts % SC;
  int lc0, lc1, lc2;
  {
    const int c = lcol < cols ? lcol % C : 0;
    lc0 = c % M0;
    lc1 = (c / M0) % M1;
    lc2 = c / (M0 * M1);
  }
  acc_t yr[RT], yi[RT];
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    yr[i] = acc_t{};
    yi[i] = acc_t{};
  }
  // The target's task descriptors sit in the lanes of every wave, 64 at a time (task base + l in
  // lane l), and are read with readlane: the cursor never waits on a memory load.
  const int nt = t.t1 - t.t0;
  int base = 0;
  int d_lo = 0, d_hi = 0, d_lda = 0, d_ks = 0, d_src = 0, d_sel = 0;
#define ML_FETCH()                                                \
  do {                                                            \
    if (base + lane < nt) {                                       \
      const MlTask w = tk[t.t0 + base + lane];                    \
      d_lo = (int)(unsigned)(w.a_off & 0xffffffffLL);             \
      d_hi = (int)(w.a_off >> 32);                                \
      d_lda = w.lda;                                              \
      d_ks = w.ks;                                                \
      d_src = w.src_row;                                          \
      d_sel = w.sel;                                              \
    }                                                             \
  } while (0)
  // items of the whole target (a wave sum per 64 tasks)
  int items = 0;
  for (base = 0; base < nt; base += 64) {
    ML_FETCH();
    items += wave_sum(base + lane < nt ? (d_ks + KW - 1) / KW : 0);
  }
  base = 0;
  if (nt > 64) ML_FETCH();  // otherwise the lanes still hold tasks 0..nt-1
  const int rounds = (items + WS - 1) / WS;
  int q = 0, ch = stream, nch = nt > 0 ? (__builtin_amdgcn_readlane(d_ks, 0) + KW - 1) / KW : 0;
  // the cursor (task q, chunk ch) of this stream moves by `by` items
#define ML_ADVANCE(by)                                                            \
  do {                                                                            \
    ch += (by);                                                                   \
    while (q < nt && ch >= nch) {                                                 \
      ch -= nch;                                                                  \
      ++q;                                                                        \
      if (q < nt && q >= base + 64) {                                             \
        base += 64;                                                               \
        ML_FETCH();                                                               \
      }                                                                           \
      nch = q < nt ? (__builtin_amdgcn_readlane(d_ks, q - base) + KW - 1) / KW : 0; \
    }                                                                             \
  } while (0)
  // the cursor's item into registers (kn = 0: no item left)
#define ML_LOAD(an, xn, kn)                                                                                        \
  do {                                                                                                   \
    kn = 0;                                                                                              \
    if (q < nt) {                                                                                        \
      const int lq = q - base;                                                                           \
      const long long a_off = (long long)(unsigned)__builtin_amdgcn_readlane(d_lo, lq) |                 \
                              ((long long)__builtin_amdgcn_readlane(d_hi, lq) << 32);                    \
      const int lda = __builtin_amdgcn_readlane(d_lda, lq);                                              \
      const int ks = __builtin_amdgcn_readlane(d_ks, lq);                                                \
      const int src_row = __builtin_amdgcn_readlane(d_src, lq);                                          \
      const int sel = __builtin_amdgcn_readlane(d_sel, lq);                                              \
      const int k0 = ch * KW;                                                                            \
      kn = min(KW, ks - k0);                                                                             \
      const cplx<T>* __restrict__ A = ops + a_off + k0;                                                  \
      _Pragma("unroll") for (int s = 0; s < STG; ++s) {                                                  \
        const int e = ts + s * SLICES * 64;                                                              \
        const int row = e / KW, kk = e % KW;                                                             \
        an[s] = load_if<T>(A + (size_t)row * lda + kk, e < ROWS * KW && row < t.rows && kk < kn);      \
      }                                                                                                  \
      const int sh = sel >> 2;                                                                           \
      const int d0 = sh % 3 - 1, d1 = (sh / 3) % 3 - 1, d2 = sh / 9 - 1;                                 \
      const int dl = d0 + M0 * (d1 + M1 * d2);                                                           \
      const cplx<T>* __restrict__ src =                                                                  \
          reinterpret_cast<const cplx<T>*>(B.b[sel & 3]) + (size_t)(src_row + k0) * cols;                \
      const bool okc = lcol < cols && (unsigned)(lc0 - d0) < (unsigned)M0 &&                             \
                       (unsigned)(lc1 - d1) < (unsigned)M1 && (unsigned)(lc2 - d2) < (unsigned)M2;        \
      _Pragma("unroll") for (int s = 0; s < XSTG; ++s) {                                                 \
        const int kk = ts / SC + 4 * s;                                                                  \
        xn[s] = load_if<T>(src + ((size_t)kk * cols + lcol - dl), okc && kk < kn);                       \
      }                                                                                                  \
    }                                                                                                    \
  } while (0)
  cplx<T> an[STG], xn[XSTG];
  int kn = 0;  // contraction length of the loaded item (0: none)
  ML_ADVANCE(0);
  ML_LOAD(an, xn, kn);
  for (int r = 0; r < rounds; ++r) {
    stream_sync<SLICES>();
#pragma unroll
    for (int s = 0; s < STG; ++s) {
      const int e = ts + s * SLICES * 64;
      if (e < ROWS * KW) As[stream][e % KW][e / KW] = an[s];
    }
#pragma unroll
    for (int s = 0; s < XSTG; ++s) {
      const int e = ts + s * SLICES * 64;
      Xs[stream][e / SC][e % SC] = xn[s];
    }
    const int kc = kn;
    ML_ADVANCE(WS);
    ML_LOAD(an, xn, kn);
    stream_sync<SLICES>();
#pragma unroll
    for (int k4 = 0; k4 < KW; k4 += 4) {
      if (k4 >= kc) break;  // uniform: the tail of the item's contraction (no item: kc = 0)
      const cplx<T> xv = Xs[stream][k4 + g][slice * 16 + li];
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const cplx<T> av = As[stream][k4 + g][16 * i + li];
        yr[i] = mf::step(av.x, xv.x, yr[i]);
        yi[i] = mf::step(av.x, xv.y, yi[i]);
        yr[i] = mf::step(-av.y, xv.y, yr[i]);
        yi[i] = mf::step(av.y, xv.x, yi[i]);
      }
    }
  }
#undef ML_LOAD
#undef ML_ADVANCE
#undef ML_FETCH
  if constexpr (WS > 1) {
    // stream j > 0 hands its partial sums to stream 0, one stream at a time (stream order)
    for (int j = 1; j < WS; ++j) {
      __syncthreads();
      if (stream == j) {
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            red[(16 * i + mf::row(g, v)) * SC + slice * 16 + li] = mk<T>(yr[i][v], yi[i][v]);
      }
      __syncthreads();
      if (stream == 0) {
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const cplx<T> o = red[(16 * i + mf::row(g, v)) * SC + slice * 16 + li];
            yr[i][v] += o.x;
            yi[i][v] += o.y;
          }
      }
    }
    if (stream > 0) return;
  }
  const int col = col0 + slice * 16 + li;
  if (col >= cols) return;
  cplx<T>* __restrict__ out = reinterpret_cast<cplx<T>*>(B.b[out_id]);
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * i + mf::row(g, v);
      if (row < t.rows) {
        cplx<T>* o = out + (size_t)(t.out_row + row) * cols + col;
        const cplx<T> a = mk<T>(yr[i][v], yi[i][v]);
        *o = accum ? cadd<T>(*o, a) : a;
      }
    }
}

// xt[pos[e]][col] = x[col][e]  (x: [R][C][n], col = r C + c)
template <typename T>
__global__ void ml_in_kernel(const cplx<T>* __restrict__ x, const int* __restrict__ pos, int n, size_t total,
                             int cols, cplx<T>* __restrict__ xt) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(i / n);
    const int e = (int)(i - (size_t)col * n);
    xt[(size_t)pos[e] * cols + col] = x[i];
  }
}

// y[col][e] (+)= yt[pos[e]][col] in the output type U (the application's precision or FP64)
template <typename T, typename U>
__global__ void ml_out_kernel(const cplx<T>* __restrict__ yt, const int* __restrict__ pos, int n, size_t total,
                              int cols, int accum, cplx<U>* __restrict__ y) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(i / n);
    const int e = (int)(i - (size_t)col * n);
    const cplx<T> v = yt[(size_t)pos[e] * cols + col];
    const cplx<U> w = mk<U>((U)v.x, (U)v.y);
    y[i] = accum ? cadd<U>(y[i], w) : w;
  }
}

// out[i] (+)= sum over slots s (in order) of part[s slot + i], i < slot
template <typename T>
__global__ void ml_reduce_kernel(const cplx<T>* __restrict__ part, int S, size_t slot, int accum,
                                 cplx<T>* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < slot; i += (size_t)gridDim.x * blockDim.x) {
    cplx<T> s = accum ? out[i] : mk<T>(0, 0);
    for (int q = 0; q < S; ++q) s = cadd<T>(s, part[(size_t)q * slot + i]);
    out[i] = s;
  }
}

// grid[bin(c)][r][i] = sum over chunks q (in order) of part[q p + i][r C + c]: a workgroup takes 64
// consecutive outputs (i, col) of the [p][cols] layout, each of its 4 waves a contiguous quarter of
// the chunks; the quarters are added in order through LDS
template <typename T>
__global__ __launch_bounds__(256) void ml_s2m_reduce_kernel(const cplx<T>* __restrict__ part, int chunks, int p,
                                                            int cols, int C, int R, int M0, int M1, int N0, int N1,
                                                            cplx<T>* __restrict__ grid) {
  __shared__ cplx<T> qs[3][64];
  const size_t total = (size_t)p * cols;
  const size_t idx = (size_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int wv = threadIdx.x >> 6;
  const int q0 = (int)((long long)chunks * wv / 4), q1 = (int)((long long)chunks * (wv + 1) / 4);
  cplx<T> s = mk<T>(0, 0);
  if (idx < total) {
#pragma unroll 8
    for (int q = q0; q < q1; ++q) s = cadd<T>(s, part[(size_t)q * total + idx]);
  }
  if (wv > 0) qs[wv - 1][threadIdx.x & 63] = s;
  __syncthreads();
  if (wv > 0 || idx >= total) return;
  for (int w = 0; w < 3; ++w) s = cadd<T>(s, qs[w][threadIdx.x]);
  const int i = (int)(idx / cols), col = (int)(idx - (size_t)i * cols);
  const int r = col / C, c = col - r * C;
  const int c0 = c % M0, c1 = (c / M0) % M1, c2 = c / (M0 * M1);
  const size_t bin = (size_t)c0 + (size_t)N0 * (c1 + (size_t)N1 * c2);
  grid[(bin * R + r) * p + i] = s;
}

// out[i][t] = in[i][perm[t]] (V0 with its columns in tree order)
__global__ void ml_permute_kernel(const double2* __restrict__ in, const int* __restrict__ perm, int rows, int n,
                                  double2* __restrict__ out) {
  const size_t total = (size_t)rows * n;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / n), t = (int)(idx - (size_t)i * n);
    out[idx] = in[(size_t)i * n + perm[t]];
  }
}

static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

size_t ml_workspace_bytes_per_rhs(const Plan& P, int precision) {
  if (!P.ml) return 0;
  const size_t el = precision == FMBEM_FP32 ? sizeof(float2) : sizeof(double2);
  return 2 * al256((size_t)P.n * P.C * el) + 2 * al256((size_t)P.ml->rows * P.C * el) +
         al256((size_t)P.ml->s2m_chunks * P.p * P.C * el) + al256(P.ml->part_rows * P.C * el) +
         al256(P.ml->p2p_part_rows * P.C * el);
}

template <typename T>
static MlBufs ml_bufs(const Plan& P, int R, void* ws) {
  const MlData& M = *P.ml;
  const int cols = R * P.C;
  const size_t el = sizeof(cplx<T>);
  char* w = reinterpret_cast<char*>(ws);
  MlBufs B;
  const size_t sz[7] = {(size_t)P.n * cols,       (size_t)M.rows * cols, (size_t)M.rows * cols, (size_t)P.n * cols,
                        (size_t)M.s2m_chunks * P.p * cols, M.part_rows * cols,  M.p2p_part_rows * cols};
  for (int i = 0; i < 7; ++i) {
    B.b[i] = w;
    w += al256(sz[i] * el);
  }
  return B;
}

template <typename T, int WS, int RT>
static void ml_stage_launch(const MlStage& st, const cplx<T>* ops, const MlBufs& B, int cols, const Plan& P,
                            hipStream_t s) {
  const int tile = 16 * (4 / WS);
  constexpr int KW = sizeof(T) == 8 ? 8 : 16;
  hipLaunchKernelGGL((ml_kernel<T, WS, RT, KW>), dim3(st.n_tg, (cols + tile - 1) / tile), dim3(256), 0, s, st.tg, st.tk,
                     ops, B, st.out, st.accum, cols, P.C, P.grid[0], P.grid[1], P.grid[2]);
}

// waves per column slice by the column count, row tiles by the stage's largest target
template <typename T, int WS>
static void ml_stage_rows(const MlStage& st, const cplx<T>* ops, const MlBufs& B, int cols, const Plan& P,
                          hipStream_t s) {
  if (st.max_rows <= 16) ml_stage_launch<T, WS, 1>(st, ops, B, cols, P, s);
  else if (st.max_rows <= 32) ml_stage_launch<T, WS, 2>(st, ops, B, cols, P, s);
  else ml_stage_launch<T, WS, 4>(st, ops, B, cols, P, s);
}

template <typename T>
static void ml_stage_any(const MlStage& st, const cplx<T>* ops, const MlBufs& B, int cols, const Plan& P,
                         hipStream_t s) {
  if (st.n_tg == 0) return;
  if (cols > 32) ml_stage_rows<T, 1>(st, ops, B, cols, P, s);
  else if (cols > 16) ml_stage_rows<T, 2>(st, ops, B, cols, P, s);
  else ml_stage_rows<T, 4>(st, ops, B, cols, P, s);
  if (st.split > 1) {
    const size_t slot = (size_t)st.nrows * cols;
    hipLaunchKernelGGL(ml_reduce_kernel<T>, dim3((unsigned)std::min<size_t>((slot + 255) / 256, 4096)), dim3(256), 0,
                       s, reinterpret_cast<const cplx<T>*>(B.b[st.part]), st.split, slot, st.dest_accum,
                       reinterpret_cast<cplx<T>*>(B.b[st.dest]) + (size_t)st.row0 * cols);
  }
}

// the input in tree order (parts & 1) and, with a far field, the S2M into the padded grid (parts & 2)
template <typename T>
hipError_t ml_prepare(const Plan& P, int R, const void* x, void* ws, void* grid, hipStream_t s, int parts) {
  const MlData& M = *P.ml;
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const int cols = R * P.C;
  const MlBufs B = ml_bufs<T>(P, R, ws);
  const size_t total = (size_t)P.n * cols;
  const unsigned g = (unsigned)std::min<size_t>((total + 255) / 256, 8192);
  if (parts & 1)
    hipLaunchKernelGGL(ml_in_kernel<T>, dim3(g), dim3(256), 0, s, reinterpret_cast<const cplx<T>*>(x), M.pos, P.n,
                       total, cols, reinterpret_cast<cplx<T>*>(B.b[0]));
  if ((parts & 2) && P.n_far > 0) {
    ml_stage_any<T>(M.s2m, reinterpret_cast<const cplx<T>*>(M.ops[prec]), B, cols, P, s);
    const size_t pt = (size_t)P.p * cols;
    hipLaunchKernelGGL(ml_s2m_reduce_kernel<T>, dim3((unsigned)((pt + 63) / 64)), dim3(256), 0, s,
                       reinterpret_cast<const cplx<T>*>(B.b[4]), M.s2m_chunks, P.p, cols, P.C, R, P.grid[0],
                       P.grid[1], P.fft[0], P.fft[1], reinterpret_cast<cplx<T>*>(grid));
  }
  return hipGetLastError();
}

// the near field from the input in tree order (ml_prepare earlier on the stream), in parts: the exact
// leaf blocks into the tree-ordered output (parts & 4); the tree stages up to the locals of the
// leaves (parts & 1); the L2P added to the output (parts & 8, after parts 4 and 1); y (+)= that
// output (parts & 2)
template <typename T>
hipError_t ml_apply(const Plan& P, int R, void* y, void* y64, void* ws, bool accum, hipStream_t s, int parts) {
  const MlData& M = *P.ml;
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const int cols = R * P.C;
  const MlBufs B = ml_bufs<T>(P, R, ws);
  const size_t total = (size_t)P.n * cols;
  const unsigned g = (unsigned)std::min<size_t>((total + 255) / 256, 8192);
  const cplx<T>* ops = reinterpret_cast<const cplx<T>*>(M.ops[prec]);
  if (parts & 4) ml_stage_any<T>(M.p2p, ops, B, cols, P, s);
  if (parts & 1)
    for (size_t i = 0; i + 1 < M.stages.size(); ++i) ml_stage_any<T>(M.stages[i], ops, B, cols, P, s);
  if (parts & 8) ml_stage_any<T>(M.stages.back(), ops, B, cols, P, s);
  if (!(parts & 2)) return hipGetLastError();
  if (y64)
    hipLaunchKernelGGL((ml_out_kernel<T, double>), dim3(g), dim3(256), 0, s,
                       reinterpret_cast<const cplx<T>*>(B.b[3]), M.pos, P.n, total, cols, accum ? 1 : 0,
                       reinterpret_cast<double2*>(y64));
  else
    hipLaunchKernelGGL((ml_out_kernel<T, T>), dim3(g), dim3(256), 0, s, reinterpret_cast<const cplx<T>*>(B.b[3]),
                       M.pos, P.n, total, cols, accum ? 1 : 0, reinterpret_cast<cplx<T>*>(y));
  return hipGetLastError();
}

template hipError_t ml_prepare<double>(const Plan&, int, const void*, void*, void*, hipStream_t, int);
template hipError_t ml_prepare<float>(const Plan&, int, const void*, void*, void*, hipStream_t, int);
template hipError_t ml_apply<double>(const Plan&, int, void*, void*, void*, bool, hipStream_t, int);
template hipError_t ml_apply<float>(const Plan&, int, void*, void*, void*, bool, hipStream_t, int);

// ---------------------------------------------------------------------------
// host: translation matrices
// ---------------------------------------------------------------------------
// I_l^mu (regular) or O_l^mu (singular) at v for l <= L: out[l l + l + mu]
static void harmonics_at(const double* v, double k, int L, bool singular, std::vector<double2>& out) {
  out.assign((size_t)(L + 1) * (L + 1), make_double2(0, 0));
  const double rho2 = v[0] * v[0] + v[1] * v[1];
  const double r = std::sqrt(rho2 + v[2] * v[2]);
  const double rho = std::sqrt(rho2);
  const double ct = v[2] / r, st = rho / r;
  const double cp = rho > 0 ? v[0] / rho : 1.0, sp = rho > 0 ? v[1] / rho : 0.0;
  std::vector<double> jl(L + 2), yl(L + 2), Nl(L + 2);
  sph_j_all(L, k * r, jl.data());
  if (singular) sph_y_all(L, k * r, yl.data());
  for (int mu = 0; mu <= L; ++mu) {
    legendre_N_col(mu, L, ct, st, Nl.data());
    const double er = std::cos(mu * std::atan2(sp, cp)), ei = std::sin(mu * std::atan2(sp, cp));
    const double sg = (mu & 1) ? -1.0 : 1.0;
    for (int l = mu; l <= L; ++l) {
      const double2 h = make_double2(jl[l], singular ? yl[l] : 0.0);
      // Y_l^mu = (-1)^mu N e^{i mu phi}; Y_l^{-mu} = N e^{-i mu phi}
      out[l * l + l + mu] = cmul<double>(h, make_double2(sg * Nl[l] * er, sg * Nl[l] * ei));
      if (mu > 0) out[l * l + l - mu] = cmul<double>(h, make_double2(Nl[l] * er, -Nl[l] * ei));
    }
  }
}

// sparse table of one translation kind: entry (row, col) = sum coef * H[hidx]
struct TransTable {
  std::vector<int> ptr, hidx;
  std::vector<double2> coef;
};

// kind 0: M2M, 1: L2L (regular harmonics); 2: M2L (singular)
static void trans_table(int nt, int kind, TransTable& T) {
  const int p = (nt + 1) * (nt + 1);
  const int L = 2 * nt;
  std::vector<double> gx, gw, tab;
  gauss_legendre_host(2 * nt + 2, gx, gw);
  theta_table(L, gx, tab);
  const int q = (int)gx.size(), W = 2 * L + 1;
  auto yt = [&](int l, int mu) { return &tab[((size_t)l * W + (L + mu)) * q]; };
  auto gaunt = [&](int a, int al, int b, int be, int c, int ga) {
    const double *x = yt(a, al), *y = yt(b, be), *z = yt(c, ga);
    double g = 0.0;
    for (int i = 0; i < q; ++i) g += gw[i] * x[i] * y[i] * z[i];
    return 0.5 * g;
  };
  static const double ire[4] = {1, 0, -1, 0}, iim[4] = {0, 1, 0, -1};
  T.ptr.assign((size_t)p * p + 1, 0);
  T.hidx.clear();
  T.coef.clear();
  for (int n = 0; n <= nt; ++n)
    for (int m = -n; m <= n; ++m)
      for (int n2 = 0; n2 <= nt; ++n2)
        for (int m2 = -n2; m2 <= n2; ++m2) {
          const int e = (n * n + n + m) * p + (n2 * n2 + n2 + m2);
          // order of the harmonic and the sign / power conventions of each kind
          const int mu = kind == 0 ? m2 - m : (kind == 1 ? m - m2 : m + m2);
          int lo = std::max(std::abs(mu), std::abs(n - n2));
          if ((n + n2 - lo) & 1) ++lo;
          for (int l = lo; l <= n + n2; l += 2) {
            double g, sgn;
            int pw;
            if (kind == 0) {
              g = gaunt(n2, -m2, n, m, l, mu);
              sgn = (m2 & 1) ? -1.0 : 1.0;
              pw = n2 - n + l;
            } else if (kind == 1) {
              g = gaunt(n, -m, n2, m2, l, mu);
              sgn = (m & 1) ? -1.0 : 1.0;
              pw = n - n2 + l;
            } else {
              g = gaunt(n, m, n2, m2, l, -mu);
              sgn = ((m + m2) & 1) ? -1.0 : 1.0;
              pw = n - n2 + l;
            }
            if (g == 0.0) continue;
            const double f = (2.0 * n2 + 1.0) * sgn * (2.0 * l + 1.0) * g;
            const int ip = ((pw % 4) + 4) % 4;
            T.coef.push_back(make_double2(f * ire[ip], f * iim[ip]));
            T.hidx.push_back(l * l + l + mu);
          }
          T.ptr[e + 1] = (int)T.coef.size();
        }
}

// matrix (row-major p x p) of a table at vector v, scaled: out[i][j] = rs[n(i)] T[i][j] cs[n(j)]
static void trans_matrix(const TransTable& T, int nt, const double* v, double k, bool singular,
                         const std::vector<double>& rs, const std::vector<double>& cs, double2* out) {
  const int p = (nt + 1) * (nt + 1);
  std::vector<double2> H;
  harmonics_at(v, k, 2 * nt, singular, H);
  std::vector<int> nof(p);
  for (int n = 0; n <= nt; ++n)
    for (int m = -n; m <= n; ++m) nof[n * n + n + m] = n;
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      const int e = i * p + j;
      double2 a = make_double2(0, 0);
      for (int t = T.ptr[e]; t < T.ptr[e + 1]; ++t) a = cadd<double>(a, cmul<double>(T.coef[t], H[T.hidx[t]]));
      const double f = rs[nof[i]] * cs[nof[j]];
      out[e] = make_double2(a.x * f, a.y * f);
    }
}

// ---------------------------------------------------------------------------
// host: tree, interaction lists, launch tables
// ---------------------------------------------------------------------------
static uint32_t morton(const int* c, int L) {
  uint32_t key = 0;
  for (int b = L - 1; b >= 0; --b)
    for (int a = 2; a >= 0; --a) key = (key << 1) | ((c[a] >> b) & 1);
  return key;
}

// every centroid inside the cell's lattice box and off the centre of its leaf (where the L2P
// gradient has no spherical-coordinate form)
bool ml_cell_fits(const std::vector<double>& geo, int n, const double pitch[3], int L) {
  for (int e = 0; e < n; ++e) {
    double dist2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double x = geo[(size_t)e * 18 + 9 + a];
      if (!(std::fabs(x) <= 0.5 * pitch[a])) return false;
      const double h = pitch[a] / (1 << L);
      const int c = std::min(std::max((int)std::floor((x + 0.5 * pitch[a]) / h), 0), (1 << L) - 1);
      const double dc = x - (-0.5 * pitch[a] + (c + 0.5) * h);
      dist2 += dc * dc;
    }
    if (!(dist2 > 1e-24 * (pitch[0] * pitch[0] + pitch[1] * pitch[1] + pitch[2] * pitch[2]))) return false;
  }
  return true;
}

hipError_t ml_build(Plan& P, const std::vector<double>& geo, hipStream_t s) {
  MlData& M = *P.ml;
  const int n = P.n, L = M.levels, nt = M.order, p = M.p;
  const bool want32 = (P.precisions & (1u << FMBEM_FP32)) != 0;
  // leaf coordinates and the tree order of the elements (Morton order of the leaves)
  std::vector<std::array<int, 3>> leafc(n);
  std::vector<uint32_t> key(n);
  const int nl = 1 << L;
  for (int e = 0; e < n; ++e) {
    for (int a = 0; a < 3; ++a) {
      const double h = P.pitch[a] / nl;
      int c = (int)std::floor((geo[(size_t)e * 18 + 9 + a] + 0.5 * P.pitch[a]) / h);
      leafc[e][a] = std::min(std::max(c, 0), nl - 1);
    }
    key[e] = morton(leafc[e].data(), L);
  }
  std::vector<int> perm(n), pos(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return key[a] < key[b]; });
  for (int t = 0; t < n; ++t) pos[perm[t]] = t;
  // boxes per level (1..L) in Morton order: coordinates, parent, children, leaf element ranges
  struct Box {
    int c[3];
    int parent = -1;
    std::vector<int> child;
    int e0 = 0, e1 = 0;  // leaves: tree positions
  };
  std::vector<std::vector<Box>> lv(L + 1);
  lv[0].resize(1);
  for (int l = 1; l <= L; ++l) {
    uint32_t last = 0xffffffffu;
    for (int t = 0; t < n; ++t) {
      const uint32_t kk = key[perm[t]] >> (3 * (L - l));
      if (kk != last) {
        Box b;
        for (int a = 0; a < 3; ++a) b.c[a] = leafc[perm[t]][a] >> (L - l);
        b.e0 = t;
        lv[l].push_back(b);
        last = kk;
      }
      lv[l].back().e1 = t + 1;
    }
  }
  for (int l = 1; l <= L; ++l) {
    // parents: boxes of level l - 1 in the same Morton order, matched by coordinates
    std::map<std::tuple<int, int, int>, int> idx;
    for (int b = 0; b < (int)lv[l - 1].size(); ++b)
      idx[{lv[l - 1][b].c[0], lv[l - 1][b].c[1], lv[l - 1][b].c[2]}] = b;
    for (int b = 0; b < (int)lv[l].size(); ++b) {
      Box& x = lv[l][b];
      const int pa = l == 1 ? 0 : idx.at({x.c[0] >> 1, x.c[1] >> 1, x.c[2] >> 1});
      x.parent = pa;
      lv[l - 1][pa].child.push_back(b);
    }
  }
  std::vector<int> base(L + 2, 0);  // first expansion row of every level (levels 1..L)
  for (int l = 1; l <= L; ++l) base[l + 1] = base[l] + (int)lv[l].size() * p;
  M.rows = base[L + 1];
  auto row0 = [&](int l, int b) { return base[l] + b * p; };
  M.boxes = base[L + 1] / p;
  M.leaves = (int)lv[L].size();
  // interaction lists: descend from the cell pairs of the near offsets
  struct Pair {
    int l, a, b, sd, tr;
  };
  std::vector<Pair> m2l, p2p;
  std::map<std::tuple<int, int, int, int>, int> tr_index;  // (level, grid offset) -> M2L matrix
  std::vector<std::tuple<int, int, int, int>> tr_list;
  std::vector<int> near;
  int rr[3];
  for (int a = 0; a < 3; ++a) rr[a] = P.grid[a] > 1 ? 1 : 0;
  std::function<void(int, int, int, const int*, int)> visit = [&](int l, int a, int b, const int* d, int sd) {
    const Box& A = lv[l][a];
    const Box& Bx = lv[l][b];
    int del[3], cheb = 0;
    for (int x = 0; x < 3; ++x) {
      del[x] = (l == 0 ? 0 : A.c[x] - Bx.c[x]) + d[x] * (1 << l);
      cheb = std::max(cheb, std::abs(del[x]));
    }
    if (cheb >= 2) {
      const auto kk = std::make_tuple(l, del[0], del[1], del[2]);
      auto it = tr_index.find(kk);
      int ti;
      if (it == tr_index.end()) {
        ti = (int)tr_list.size();
        tr_index[kk] = ti;
        tr_list.push_back(kk);
      } else {
        ti = it->second;
      }
      m2l.push_back(Pair{l, a, b, sd, ti});
      return;
    }
    if (l == L) {
      p2p.push_back(Pair{l, a, b, sd, -1});
      return;
    }
    for (int ca : A.child)
      for (int cb : Bx.child) visit(l + 1, ca, cb, d, sd);
  };
  for (int d2 = -rr[2]; d2 <= rr[2]; ++d2)
    for (int d1 = -rr[1]; d1 <= rr[1]; ++d1)
      for (int d0 = -rr[0]; d0 <= rr[0]; ++d0) {
        const int d[3] = {d0, d1, d2};
        visit(0, 0, 0, d, (d0 + 1) + 3 * (d1 + 1) + 9 * (d2 + 1));
      }
  M.m2l_pairs = (long long)m2l.size();
  M.p2p_pairs = (long long)p2p.size();
  // operator pool: [V p x n][U n x p][M2M (L-1) x 8][L2L (L-1) x 8][M2L][P2P blocks]
  const long long pp = (long long)p * p;
  const long long oV = 0, oU = (long long)p * n, oM = oU + (long long)n * p;
  const long long oL = oM + (long long)std::max(L - 1, 0) * 8 * pp;
  const long long oK = oL + (long long)std::max(L - 1, 0) * 8 * pp;
  const long long oP = oK + (long long)tr_list.size() * pp;
  std::vector<long long> poff(p2p.size());
  long long pe = 0;
  for (size_t i = 0; i < p2p.size(); ++i) {
    const Box& A = lv[L][p2p[i].a];
    const Box& Bx = lv[L][p2p[i].b];
    poff[i] = pe;
    pe += (long long)(A.e1 - A.e0) * (Bx.e1 - Bx.e0);
  }
  M.p2p_entries = pe;
  M.oS = oP + pe;
  M.ops_elems = (size_t)(M.oS + (long long)P.p * n);
  M.s2m_chunks = (n + kMlS2mChunk - 1) / kMlS2mChunk;
  // algorithmic work per RHS: every stage over the cells whose source cell lies in the lattice
  {
    auto inside = [&](int sd) {
      const int d[3] = {sd % 3 - 1, (sd / 3) % 3 - 1, sd / 9 - 1};
      double c = 1.0;
      for (int a = 0; a < 3; ++a) c *= P.grid[a] - std::abs(d[a]);
      return c;
    };
    double macs = 2.0 * (double)p * n * P.C;  // P2M and L2P
    for (int l = 2; l <= L; ++l) macs += 2.0 * (double)lv[l].size() * pp * P.C;  // M2M and L2L
    for (const Pair& q : m2l) macs += (double)pp * inside(q.sd);
    for (size_t i = 0; i < p2p.size(); ++i) {
      const Box& A = lv[L][p2p[i].a];
      const Box& Bx = lv[L][p2p[i].b];
      macs += (double)(A.e1 - A.e0) * (Bx.e1 - Bx.e0) * inside(p2p[i].sd);
    }
    M.macs_per_rhs = macs;
  }
  // level scalings s_l^n
  std::vector<std::vector<double>> sig(L + 1, std::vector<double>(nt + 1)), isig = sig;
  for (int l = 0; l <= L; ++l) {
    double hd = 0.0;
    for (int a = 0; a < 3; ++a) hd += std::pow(P.pitch[a] / (1 << l), 2);
    const double sl = std::min(1.0, std::max(1e-3, P.k * 0.5 * std::sqrt(hd)));
    for (int i = 0; i <= nt; ++i) {
      sig[l][i] = std::pow(sl, i);
      isig[l][i] = 1.0 / sig[l][i];
    }
  }
  // translation matrices on the host
  std::vector<double2> hT((size_t)(oP - oM));
  {
    TransTable t0, t1, t2;
    trans_table(nt, 0, t0);
    trans_table(nt, 1, t1);
    trans_table(nt, 2, t2);
    for (int l = 2; l <= L; ++l)
      for (int oct = 0; oct < 8; ++oct) {
        double b[3];
        for (int a = 0; a < 3; ++a) {
          const double h = P.pitch[a] / (1 << l);
          b[a] = (((oct >> a) & 1) ? 0.5 : -0.5) * h;  // child centre minus parent centre
        }
        // M2M child (level l) -> parent (level l - 1): b = child - parent; moments / s^n
        trans_matrix(t0, nt, b, P.k, false, isig[l - 1], sig[l], &hT[(size_t)(((l - 2) * 8 + oct) * pp)]);
        // L2L parent -> child: b = child - parent
        trans_matrix(t1, nt, b, P.k, false, sig[l], isig[l - 1],
                     &hT[(size_t)(oL - oM + ((l - 2) * 8 + oct) * pp)]);
      }
    for (size_t i = 0; i < tr_list.size(); ++i) {
      const int l = std::get<0>(tr_list[i]);
      const int del[3] = {std::get<1>(tr_list[i]), std::get<2>(tr_list[i]), std::get<3>(tr_list[i])};
      double D[3];
      for (int a = 0; a < 3; ++a) D[a] = del[a] * (P.pitch[a] / (1 << l));
      trans_matrix(t2, nt, D, P.k, true, sig[l], sig[l], &hT[(size_t)(oK - oM + (long long)i * pp)]);
    }
  }
  // launch tables
  std::vector<MlTarget> tg;
  std::vector<MlTask> tk;
  std::vector<std::pair<int, int>> stage_range;  // first target, count
  std::vector<std::pair<int, int>> stage_mode;   // out buffer, accumulate
  std::vector<int> stage_rows;
  auto begin_stage = [&](int out, int accum) {
    stage_range.push_back({(int)tg.size(), 0});
    stage_mode.push_back({out, accum});
    stage_rows.push_back(0);
  };
  auto add_target = [&](int out_row, int rows) {
    tg.push_back(MlTarget{out_row, rows, (int)tk.size(), (int)tk.size()});
    ++stage_range.back().second;
    stage_rows.back() = std::max(stage_rows.back(), rows);
  };
  auto add_task = [&](long long a_off, int lda, int ks, int src_row, int buf, int sd) {
    tk.push_back(MlTask{a_off, lda, ks, src_row, buf | (sd << 2)});
    tg.back().t1 = (int)tk.size();
  };
  // P2M
  begin_stage(1, 0);
  for (int b = 0; b < (int)lv[L].size(); ++b) {
    const Box& x = lv[L][b];
    add_target(row0(L, b), p);
    add_task(oV + x.e0, n, x.e1 - x.e0, x.e0, 0, kMlZeroShift);
  }
  // M2M, finest parents first
  for (int l = L - 1; l >= 1; --l) {
    begin_stage(1, 0);
    for (int b = 0; b < (int)lv[l].size(); ++b) {
      add_target(row0(l, b), p);
      for (int c : lv[l][b].child) {
        const Box& x = lv[l + 1][c];
        const int oct = (x.c[0] & 1) + 2 * (x.c[1] & 1) + 4 * (x.c[2] & 1);
        add_task(oM + ((long long)(l + 1 - 2) * 8 + oct) * pp, p, p, row0(l + 1, c), 1, kMlZeroShift);
      }
    }
  }
  // M2L of every level, grouped by target box (every box gets a target, so the locals start at 0)
  {
    begin_stage(2, 0);
    std::vector<std::vector<std::vector<int>>> by(L + 1);
    for (int l = 1; l <= L; ++l) by[l].resize(lv[l].size());
    for (size_t i = 0; i < m2l.size(); ++i) by[m2l[i].l][m2l[i].a].push_back((int)i);
    for (int l = 1; l <= L; ++l)
      for (int b = 0; b < (int)lv[l].size(); ++b) {
        add_target(row0(l, b), p);
        for (int i : by[l][b]) {
          const Pair& q = m2l[i];
          add_task(oK + (long long)q.tr * pp, p, p, row0(l, q.b), 1, q.sd);
        }
      }
  }
  // L2L, coarsest children first, added to the M2L locals
  for (int l = 2; l <= L; ++l) {
    begin_stage(2, 1);
    for (int b = 0; b < (int)lv[l].size(); ++b) {
      const Box& x = lv[l][b];
      const int oct = (x.c[0] & 1) + 2 * (x.c[1] & 1) + 4 * (x.c[2] & 1);
      add_target(row0(l, b), p);
      add_task(oL + ((long long)(l - 2) * 8 + oct) * pp, p, p, row0(l - 1, x.parent), 2, kMlZeroShift);
    }
  }
  // L2P per leaf, in chunks of at most kMlLeafRows element rows, added to the P2P output
  begin_stage(3, 1);
  for (int b = 0; b < (int)lv[L].size(); ++b) {
    const Box& x = lv[L][b];
    for (int r0 = x.e0; r0 < x.e1; r0 += kMlLeafRows) {
      add_target(r0, std::min(kMlLeafRows, x.e1 - r0));
      add_task(oU + (long long)r0 * p, p, p, row0(L, b), 2, kMlZeroShift);
    }
  }
  // P2P per leaf, the same row chunks (every leaf is near itself, so every chunk has a task)
  {
    begin_stage(3, 0);
    std::vector<std::vector<int>> by(lv[L].size());
    for (size_t i = 0; i < p2p.size(); ++i) by[p2p[i].a].push_back((int)i);
    for (int b = 0; b < (int)lv[L].size(); ++b) {
      const Box& x = lv[L][b];
      for (int r0 = x.e0; r0 < x.e1; r0 += kMlLeafRows) {
        add_target(r0, std::min(kMlLeafRows, x.e1 - r0));
        for (int i : by[b]) {
          const Box& y = lv[L][p2p[i].b];
          const int ns = y.e1 - y.e0;
          add_task(oP + poff[i] + (long long)(r0 - x.e0) * ns, ns, ns, y.e0, 0, p2p[i].sd);
        }
      }
    }
  }
  // S2M of the cell-level far field (kept last; launched by ml_prepare): partial sums over element
  // chunks into buffer 4, rows q p + i
  begin_stage(4, 0);
  for (int r0 = 0; r0 < P.p; r0 += kMlRows)
    for (int q = 0; q < M.s2m_chunks; ++q) {
      const int k0 = q * kMlS2mChunk;
      add_target(q * P.p + r0, std::min(kMlRows, P.p - r0));
      add_task(M.oS + (long long)r0 * n + k0, n, std::min(kMlS2mChunk, n - k0), k0, 0, kMlZeroShift);
    }
  // stages whose targets carry many tasks (M2L, P2P) are divided over more workgroups when
  // the targets alone would leave the CUs short of work (columns of a one-RHS application).  The
  // P2P stage runs beside the tree stages, so its split hardly matters (1, 2, 4 or 8 slots within
  // 1 % on the 4 x 4 lattice of 20480-triangle cells, n_t,near = 4)
  std::vector<std::array<int, 5>> split_of(stage_range.size(), {1, 0, 0, 0, 0});  // split, dest, accum, row0, nrows
  auto split_stage = [&](size_t si, int row0s, int nrows, int part) {
    const int first = stage_range[si].first, count = stage_range[si].second;
    if (count == 0) return;
    const int tile = P.C > 32 ? 64 : (P.C > 16 ? 32 : 16);
    const long long wgs = (long long)count * ((P.C + tile - 1) / tile);
    long long tasks = 0;
    for (int i = first; i < first + count; ++i) tasks += tg[i].t1 - tg[i].t0;
    int S = (int)std::min<long long>(8, (2048 + wgs - 1) / wgs);
    S = (int)std::min<long long>(S, std::max<long long>(1, tasks / (4LL * count)));
    if (S <= 1) return;
    const int nfirst = (int)tg.size();
    for (int s2 = 0; s2 < S; ++s2)
      for (int i = first; i < first + count; ++i) {
        const MlTarget x = tg[i];
        // tasks of slot s2: a contiguous share of the target's contraction length
        long long total = 0;
        for (int q = x.t0; q < x.t1; ++q) total += tk[q].ks;
        long long acc = 0;
        int a = x.t0, b = x.t0;
        for (int q = x.t0; q < x.t1; ++q) {
          const long long mid = acc + tk[q].ks / 2;  // a task goes to the slot holding its middle
          const int owner = total > 0 ? (int)std::min<long long>(S - 1, mid * S / total) : 0;
          if (owner < s2) a = q + 1;
          if (owner <= s2) b = q + 1;
          acc += tk[q].ks;
        }
        if (b < a) b = a;
        tg.push_back(MlTarget{s2 * nrows + (x.out_row - row0s), x.rows, a, b});
      }
    stage_range[si] = {nfirst, S * count};
    split_of[si] = {S, stage_mode[si].first, stage_mode[si].second, row0s, nrows};
    stage_mode[si] = {part, 0};
    size_t& rows_of_part = part == 5 ? M.part_rows : M.p2p_part_rows;
    rows_of_part = std::max(rows_of_part, (size_t)S * nrows);
  };
  // expansion targets of more than 32 rows (p > 32) become balanced row blocks of at most 32, each
  // with the tasks' operators offset to its rows (fewer idle rows in the 32- and 64-row tiles)
  auto row_split_stage = [&](size_t si) {
    const int first = stage_range[si].first, count = stage_range[si].second;
    bool any = false;
    for (int i = first; i < first + count; ++i) any = any || tg[i].rows > 32;
    if (!any) return;
    const int nfirst = (int)tg.size();
    int maxr = 0;
    for (int i = first; i < first + count; ++i) {
      const MlTarget x = tg[i];
      const int nch = (x.rows + 31) / 32, rc = (x.rows + nch - 1) / nch;
      for (int c = 0; c < nch; ++c) {
        const int r0 = c * rc, rows = std::min(rc, x.rows - r0);
        const int t0 = (int)tk.size();
        for (int q = x.t0; q < x.t1; ++q) {
          MlTask w = tk[q];
          w.a_off += (long long)r0 * w.lda;
          tk.push_back(w);
        }
        tg.push_back(MlTarget{x.out_row + r0, rows, t0, (int)tk.size()});
        maxr = std::max(maxr, rows);
      }
    }
    stage_range[si] = {nfirst, (int)tg.size() - nfirst};
    stage_rows[si] = maxr;
  };
  {
    // stage order: P2M, M2M x (L - 1), M2L, L2L x (L - 1), L2P, P2P, S2M
    const size_t m2l_stage = 1 + (size_t)(L - 1), l2p_stage = m2l_stage + 1 + (size_t)(L - 1);
    for (size_t si = 0; si < l2p_stage; ++si) row_split_stage(si);
    split_stage(m2l_stage, 0, M.rows, 5);
    split_stage(l2p_stage + 1, 0, n, 6);
  }
  // device arrays
  hipError_t e;
  MlTarget* d_tg = nullptr;
  MlTask* d_tk = nullptr;
  if ((e = plan_alloc(P, (void**)&d_tg, std::max<size_t>(1, tg.size()) * sizeof(MlTarget)))) return e;
  if ((e = plan_alloc(P, (void**)&d_tk, std::max<size_t>(1, tk.size()) * sizeof(MlTask)))) return e;
  if ((e = plan_alloc(P, (void**)&M.pos, n * sizeof(int)))) return e;
  if ((e = plan_alloc(P, (void**)&M.perm, n * sizeof(int)))) return e;
  if ((e = plan_alloc(P, &M.ops[0], M.ops_elems * sizeof(double2)))) return e;
  if (want32 && (e = plan_alloc(P, &M.ops[1], M.ops_elems * sizeof(float2)))) return e;
  hipMemcpyAsync(d_tg, tg.data(), tg.size() * sizeof(MlTarget), hipMemcpyHostToDevice, s);
  hipMemcpyAsync(d_tk, tk.data(), tk.size() * sizeof(MlTask), hipMemcpyHostToDevice, s);
  hipMemcpyAsync(M.pos, pos.data(), n * sizeof(int), hipMemcpyHostToDevice, s);
  hipMemcpyAsync(M.perm, perm.data(), n * sizeof(int), hipMemcpyHostToDevice, s);
  double2* ops = reinterpret_cast<double2*>(M.ops[0]);
  hipMemcpyAsync(ops + oM, hT.data(), hT.size() * sizeof(double2), hipMemcpyHostToDevice, s);
  M.max_tasks = 0;
  for (size_t i = 0; i < stage_range.size(); ++i)
    for (int x = stage_range[i].first; x < stage_range[i].first + stage_range[i].second; ++x)
      M.max_tasks = std::max(M.max_tasks, tg[x].t1 - tg[x].t0);
  auto make_stage = [&](size_t i) {
    return MlStage{d_tg + stage_range[i].first, d_tk,          stage_range[i].second, stage_mode[i].first,
                   stage_mode[i].second,         stage_rows[i], split_of[i][0],        split_of[i][1],
                   split_of[i][2],               split_of[i][3], split_of[i][4],       stage_mode[i].first};
  };
  M.stages.clear();
  for (size_t i = 0; i + 2 < stage_range.size(); ++i) M.stages.push_back(make_stage(i));
  M.p2p = make_stage(stage_range.size() - 2);
  M.s2m = make_stage(stage_range.size() - 1);
  // leaf P2M / L2P about the leaf centres (device), and the exact P2P entries
  std::vector<double> cen((size_t)n * 3);
  for (int e2 = 0; e2 < n; ++e2)
    for (int a = 0; a < 3; ++a) {
      const double h = P.pitch[a] / nl;
      cen[(size_t)e2 * 3 + a] = -0.5 * P.pitch[a] + (leafc[e2][a] + 0.5) * h;
    }
  std::vector<P2pBlock> blocks(p2p.size());
  for (size_t i = 0; i < p2p.size(); ++i) {
    const Box& A = lv[L][p2p[i].a];
    const Box& Bx = lv[L][p2p[i].b];
    blocks[i] = P2pBlock{oP + poff[i], A.e0, A.e1 - A.e0, Bx.e0, Bx.e1 - Bx.e0, p2p[i].sd};
  }
  e = ml_assemble_launch(P, nt, cen, isig[L], blocks, pe, ops, oV, oU, s);
  if (!e) {
    hipLaunchKernelGGL(ml_permute_kernel, dim3(4096), dim3(256), 0, s, reinterpret_cast<const double2*>(P.V0[0]),
                       M.perm, P.p, n, ops + M.oS);
    e = hipGetLastError();
  }
  if (!e && want32) e = cast_launch(ops, reinterpret_cast<float2*>(M.ops[1]), M.ops_elems, s);
  // the host tables must outlive their copies, also when a step failed
  const hipError_t e2 = hipStreamSynchronize(s);
  return e ? e : e2;
}

}  // namespace fmbem
