// Grouped complex GEMM on the matrix cores for the dense contractions of the
// FMPBEM apply (Sec. 3.2, eq. (2dPeriodicFMM); Sec. 3.5, eq. (FMPBEMsystem)):
//
//   near field  part_d[:, (r,c)] = S_d x_{(r, c-d)}   for every near offset d  (n x n blocks)
//   S2M         mhat[bin(c)][r]  = V0 x_{(r, c)}                                (p x n, into the padded grid)
//   L2T         y[:, (r,c)]      = sum_d part_d[:, (r,c)] + U0 l[bin(c)][r]     (n x p, from the padded grid)
//
// A job is one GEMM whose B columns are the cells (x right-hand sides) of x,
// shifted by the job's cell offset, or the bins of the padded grid.  Jobs of
// different lattices (plans) can share one launch: each job carries its own
// lattice geometry.  The launch is a flat list of workgroups; workgroup w owns
// row tile w / ctiles and column tile w % ctiles of its job, and the list is dealt
// so that the column tiles of one row tile land on one XCD (the hardware deals
// consecutive workgroup ids round-robin over the 8 XCDs), where the A tile is
// read from HBM once into that XCD's L2.  The near partial products are summed in
// a fixed order in the L2T epilogue (deterministic, independent of batching).
//
// Complex products take three real products per complex product (Gauss):
//   P1 = Re A Re B,  P2 = Im A Im B,  P3 = (Re A + Im A)(Re B + Im B),
//   Re = P1 - P2,    Im = P3 - P1 - P2,
// on 16x16x4 MFMA tiles (FP32 or FP64), i.e. 3/4 of the matrix-core work of the
// 2x2 real split form.  Within one step of KC complex k, the four k slots of an
// MFMA are taken by lane group g = lane / 16 over k = g * KC/4 + t (t = 0 .. KC/4-1):
// the sum over k is the same, and every lane reads its KC/4 operands of a row or
// column with one 16-byte LDS load.  LDS holds two steps (ping-pong): the global
// loads of step s+1 are issued before the MFMAs of step s and stored after them, one
// barrier per step.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "mfma.hpp"

namespace fmbem {

__device__ inline void cell_coords(const NearJob& jb, int j, int& r, int& i1, int& i2, int& i3) {
  r = j / jb.C;
  const int c = j - r * jb.C;
  i1 = c % jb.M0;
  const int t = c / jb.M0;
  i2 = t % jb.M1;
  i3 = t / jb.M1;
}

// LDS layout of one operand tile: a row (of A) or column (of B) holds the KC k values of
// one step in four 16-byte chunks (KC = 16 floats or 8 doubles); chunk c of row r sits
// at slot 4 r + (c ^ ((r >> 2) & 3)).  The XOR makes both access patterns free of bank
// conflicts without padding: a fragment read (16 rows, one chunk each) and a staging
// write (consecutive rows, whole chunks) both touch 64 distinct banks per 16 lanes.
__device__ inline int lds_slot(int r, int c) { return 4 * r + (c ^ ((r >> 2) & 3)); }

// Tile: ROWS complex rows x COLS columns, 4 waves arranged WR x (4/WR), KC complex k per step.
// ACOL: batched job with column-major A (the M2L products).  PIPE: k steps whose global loads
// are in flight at once (1: the next step during the MFMAs of the current one; 2: also the one
// after, in a second register set).  FINAL: the kernel takes DEST_FINAL jobs (the L2T launch
// only, so that the other launches do not carry the registers of its epilogue).  JL: the job
// list; DftGemmJobs makes the tile an axis pass of the grid DFT (column-major A = the grid
// lines, product b = line b, one DFT matrix as B, in-place output, symmetry signs).
template <typename T, int ROWS, int COLS, int WR, int KC, int PIPE, bool ACOL = false, bool FINAL = false,
          typename JL = NearJobs>
__device__ __forceinline__ void near_tile(const JL& jobs) {
  constexpr bool DFTG = std::is_same<JL, DftGemmJobs>::value;
  static_assert(!DFTG || ACOL, "the DFT passes use the column-major A form");
  constexpr int WC = 4 / WR;
  constexpr int RBW = ROWS / (16 * WR);  // 16-row MFMA blocks per wave
  constexpr int CBW = COLS / (16 * WC);  // 16-column MFMA blocks per wave
  static_assert(RBW >= 1 && CBW >= 1 && RBW * 16 * WR == ROWS && CBW * 16 * WC == COLS, "tile / wave grid");
  constexpr int CW = 16 / sizeof(T);            // values per 16-byte chunk
  static_assert(KC * sizeof(T) == 64, "one step = four 16-byte chunks per row");
  constexpr int AT = ROWS * KC;                 // A complex elements per step
  constexpr int APT = AT >= 256 ? AT / 256 : 1; // per thread (consecutive k)
  constexpr int BPT = COLS * KC / 256;          // B complex elements per thread (consecutive k)
  constexpr int TPC = KC / BPT;                 // threads per B column
  static_assert(BPT >= 1 && KC % BPT == 0 && (BPT % CW == 0 || CW % BPT == 0), "B staging split");
  static_assert(ACOL ? ROWS % APT == 0 : (KC % APT == 0 && (APT % CW == 0 || CW % APT == 0)), "A staging split");
  typedef T VK __attribute__((ext_vector_type(CW)));
  // two buffers (ping-pong over the k steps) x {Re, Im} of A and of B, in chunks; the
  // sums Re + Im of the third product are formed in registers after the fragment loads
  // one LDS block: the operand buffers during the k loop, the output tile in the epilogue
  __shared__ VK Ops[2 * 2 * (ROWS + COLS) * 4];
  auto Asm = [&](int b, int c) -> VK* { return Ops + ((b * 2 + c) * (ROWS + COLS)) * 4; };
  auto Bsm = [&](int b, int c) -> VK* { return Ops + ((b * 2 + c) * (ROWS + COLS) + ROWS) * 4; };
  using Acc = typename nmf<T>::acc;

  // logical workgroup (XCD-aware deal), job and tile
  int L = (int)blockIdx.x;
  {
    const int per = jobs.total / 8;
    if (L < per * 8) L = (L % 8) * per + L / 8;
  }
  int ji = 0;
  while (ji + 1 < jobs.count && L >= jobs.job[ji + 1].tile0) ++ji;
  const NearJob& jb = jobs.job[ji];
  const int M = jb.M, K = jb.K, N = jb.N, lda = jb.lda;
  const int ctiles = (N + COLS - 1) / COLS;
  int local = L - jb.tile0;
  int bb = 0;  // product of a batched job
  if constexpr (ACOL) {
    const int per = ((M + ROWS - 1) / ROWS) * ctiles;
    bb = local / per;
    local -= bb * per;
  }
  const int m0 = (local / ctiles) * ROWS;
  const int col0 = (local % ctiles) * COLS;
  // DFT pass: line bb = (u, v) of the pass starts at u su + v sv
  long long line_off = 0;
  int line_u = 0, line_v = 0;
  if constexpr (DFTG) {
    line_u = bb % jobs.dg.U;
    line_v = bb / jobs.dg.U;
    line_off = line_u * jobs.dg.su + line_v * jobs.dg.sv;
  }
  const cplx<T>* A = reinterpret_cast<const cplx<T>*>(jb.A) +
                     (DFTG ? (size_t)line_off : ACOL ? (size_t)(jb.amap ? jb.amap[bb] : bb) * K * lda : 0);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int g = lane >> 4, li = lane & 15;

  // B column of this thread; nullptr = zero column (shifted outside the lattice)
  const int b_col = tid / TPC;
  const int b_k = (tid % TPC) * BPT;
  const cplx<T>* bcol = nullptr;
  {
    const int j = col0 + b_col;
    if (j < N) {
      int r, i1, i2, i3;
      cell_coords(jb, j, r, i1, i2, i3);
      const cplx<T>* src = reinterpret_cast<const cplx<T>*>(jb.src);
      if (DFTG) {
        bcol = src + (size_t)j * K;  // one DFT matrix for every line
      } else if (ACOL) {
        bcol = src + ((size_t)bb * N + j) * K;
      } else if (jb.src_kind == SRC_X) {
        const int s1 = i1 - jb.d0, s2 = i2 - jb.d1, s3 = i3 - jb.d2;
        if (s1 >= 0 && s1 < jb.M0 && s2 >= 0 && s2 < jb.M1 && s3 >= 0 && s3 < jb.M2)
          bcol = src + ((size_t)r * jb.C + (s1 + jb.M0 * (s2 + jb.M1 * s3))) * K;
      } else {
        const size_t bin = (size_t)i1 + (size_t)jb.N0 * (i2 + (size_t)jb.N1 * i3);
        bcol = src + (bin * jb.R + r) * K;
      }
    }
  }
  // A staging: thread t < AT / APT holds APT consecutive k of one row (row-major A) or
  // APT consecutive rows of one k (column-major A)
  const bool a_act = tid * APT < AT;
  const int a_row = ACOL ? (tid * APT) % ROWS : (tid * APT) / KC;
  const int a_k = ACOL ? (tid * APT) / ROWS : (tid * APT) % KC;
  const cplx<T>* arow = (!ACOL && a_act && m0 + a_row < M) ? A + (size_t)(m0 + a_row) * lda : nullptr;

  Acc p1[RBW][CBW], p2[RBW][CBW], p3[RBW][CBW];
#pragma unroll
  for (int i = 0; i < RBW; ++i)
#pragma unroll
    for (int j = 0; j < CBW; ++j) {
      p1[i][j] = Acc{0, 0, 0, 0};
      p2[i][j] = Acc{0, 0, 0, 0};
      p3[i][j] = Acc{0, 0, 0, 0};
    }

  // staged global loads, one register set per step in flight
  cplx<T> ra2[PIPE][APT];
  cplx<T> rb2[PIPE][BPT];
  uint32_t amask2[PIPE], bmask2[PIPE];  // valid staged elements (bit q); invalid ones are stored as zero
  // Global loads of one step, branch-free: every load reads a valid address (out-of-range
  // rows, columns and k read a valid stand-in, masked to zero at the LDS store), so the
  // loads stay in flight across the MFMAs of the current step.  When K is a multiple of
  // the 16-byte unit (two FP32 or one FP64 complex value), whole units are loaded; in the
  // column-major form (batched products) the A columns are loaded in whole units when the
  // column stride lda is a multiple of the unit, and the B columns element by element.
  constexpr int EPL = 16 / sizeof(cplx<T>);
  using VL = typename Vec16<T>::type;
  const bool vec_ok = ACOL ? (lda % EPL) == 0 && (reinterpret_cast<uintptr_t>(jb.A) % 16) == 0 : (K % EPL) == 0;
  const bool a_in = !ACOL && a_act && m0 + a_row < M;
  const cplx<T>* arow_ld = A + (size_t)(a_in ? m0 + a_row : 0) * lda;
  // column-major A: valid rows of this thread's APT (bit q), and the column offset of its k
  // (threads without a k of the step read column k0 of the step, masked)
  uint32_t acol_rows = 0;
  if constexpr (ACOL) {
#pragma unroll
    for (int q = 0; q < APT; ++q) acol_rows |= ((a_act && m0 + a_row + q < M) ? 1u : 0u) << q;
  }
  const int a_k_ld = a_act ? a_k : 0;
  const bool b_in = bcol != nullptr;
  const cplx<T>* bcol_ld = b_in ? bcol : reinterpret_cast<const cplx<T>*>(jb.src);
  auto unpack = [](const VL& v, cplx<T>* r) {
    if constexpr (EPL == 2) {
      r[0] = mk<T>(v.x, v.y);
      r[1] = mk<T>(v.z, v.w);
    } else {
      r[0] = mk<T>(v.x, v.y);
    }
  };
  // full step (k0 + KC <= K): whole 16-byte units, no per-step address or mask arithmetic
  auto load_full = [&](int k0, auto set) {
    cplx<T>* ra = ra2[decltype(set)::value];
    cplx<T>* rb = rb2[decltype(set)::value];
    uint32_t& amask = amask2[decltype(set)::value];
    uint32_t& bmask = bmask2[decltype(set)::value];
    if constexpr (ACOL) {
      // a unit starting at row r < lda lies inside the column (r and lda multiples of EPL);
      // units from row lda on read row 0 of the column instead (masked)
      const cplx<T>* acol = A + (size_t)(k0 + a_k_ld) * lda;
#pragma unroll
      for (int q = 0; q < APT / EPL; ++q) {
        const int r = m0 + a_row + q * EPL;
        unpack(*reinterpret_cast<const VL*>(acol + (r < lda ? r : 0)), ra + q * EPL);
      }
      amask = acol_rows;
#pragma unroll
      for (int e = 0; e < BPT; ++e) rb[e] = bcol_ld[k0 + b_k + e];
    } else {
#pragma unroll
      for (int q = 0; q < APT / EPL; ++q)
        unpack(*reinterpret_cast<const VL*>(arow_ld + k0 + a_k + q * EPL), ra + q * EPL);
      amask = a_in ? 0xFFFFFFFFu : 0u;
#pragma unroll
      for (int q = 0; q < BPT / EPL; ++q)
        unpack(*reinterpret_cast<const VL*>(bcol_ld + k0 + b_k + q * EPL), rb + q * EPL);
    }
    bmask = b_in ? 0xFFFFFFFFu : 0u;
  };
  // any step: element loads from clamped indices, per-element masks
  auto load_any = [&](int k0, auto set) {
    cplx<T>* ra = ra2[decltype(set)::value];
    cplx<T>* rb = rb2[decltype(set)::value];
    uint32_t& amask = amask2[decltype(set)::value];
    uint32_t& bmask = bmask2[decltype(set)::value];
    amask = 0;
    if (ACOL) {
      const bool kin = a_act && k0 + a_k < K;
      const cplx<T>* acol = A + (size_t)(kin ? k0 + a_k : 0) * lda + m0 + a_row;
#pragma unroll
      for (int q = 0; q < APT; ++q) {
        const bool v = kin && m0 + a_row + q < M;
        ra[q] = v ? acol[q] : mk<T>(0, 0);
        amask |= (v ? 1u : 0u) << q;
      }
      if constexpr (DFTG) {
        // first inverse pass: the factor D leaves the non-canonical bins on the way in
        const DftFlip& fl = jobs.dg.flip;
        if (fl.mode == 2 && kin && bin_flipped(fl, k0 + a_k, line_u, line_v)) {
#pragma unroll
          for (int q = 0; q < APT; ++q)
            if (odd_degree(m0 + a_row + q, fl.p)) ra[q] = mk<T>(-ra[q].x, -ra[q].y);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < APT; ++q) {
        const int kk = k0 + a_k + q;
        const bool v = a_in && kk < K;
        ra[q] = arow_ld[v ? kk : 0];
        amask |= (v ? 1u : 0u) << q;
      }
    }
    bmask = 0;
#pragma unroll
    for (int e = 0; e < BPT; ++e) {
      const int kk = k0 + b_k + e;
      const bool v = b_in && kk < K;
      rb[e] = bcol_ld[v ? kk : 0];
      bmask |= (v ? 1u : 0u) << e;
    }
  };
  // the full-step path needs 16-byte aligned rows / columns and whole units per thread (the DFT
  // passes keep the element loads, which apply the symmetry signs)
  constexpr bool kVecShape = ACOL ? (!DFTG && APT % EPL == 0) : (APT % EPL == 0 && BPT % EPL == 0);
  const bool vec_steps = kVecShape && vec_ok;
  // staged values of a register set -> LDS buffer b (whole chunks as one 16-byte store, partial
  // chunks element-wise)
  auto store = [&](int b, auto set) {
    const cplx<T>* ra = ra2[decltype(set)::value];
    const cplx<T>* rb = rb2[decltype(set)::value];
    const uint32_t amask = amask2[decltype(set)::value], bmask = bmask2[decltype(set)::value];
    auto av = [&](int q, T x) { return ((amask >> q) & 1u) ? x : T(0); };
    auto bv = [&](int q, T x) { return ((bmask >> q) & 1u) ? x : T(0); };
    if (ACOL) {
      if (a_act) {
        // APT rows of one k: element-wise into their rows' chunks
        const int c = a_k / CW, w = a_k % CW;
#pragma unroll
        for (int q = 0; q < APT; ++q) {
          const int o = lds_slot(a_row + q, c);
          reinterpret_cast<T*>(&Asm(b, 0)[o])[w] = av(q, ra[q].x);
          reinterpret_cast<T*>(&Asm(b, 1)[o])[w] = av(q, ra[q].y);
        }
      }
    } else if (a_act) {
      if constexpr (APT >= CW) {
#pragma unroll
        for (int c = 0; c < APT / CW; ++c) {
          VK vr, vi;
#pragma unroll
          for (int e = 0; e < CW; ++e) {
            vr[e] = av(c * CW + e, ra[c * CW + e].x);
            vi[e] = av(c * CW + e, ra[c * CW + e].y);
          }
          const int o = lds_slot(a_row, a_k / CW + c);
          Asm(b, 0)[o] = vr;
          Asm(b, 1)[o] = vi;
        }
      } else {
        const int o = lds_slot(a_row, a_k / CW);
        T* pr = reinterpret_cast<T*>(&Asm(b, 0)[o]) + a_k % CW;
        T* pi = reinterpret_cast<T*>(&Asm(b, 1)[o]) + a_k % CW;
#pragma unroll
        for (int q = 0; q < APT; ++q) {
          pr[q] = av(q, ra[q].x);
          pi[q] = av(q, ra[q].y);
        }
      }
    }
    if constexpr (BPT >= CW) {
#pragma unroll
      for (int c = 0; c < BPT / CW; ++c) {
        VK vr, vi;
#pragma unroll
        for (int e = 0; e < CW; ++e) {
          vr[e] = bv(c * CW + e, rb[c * CW + e].x);
          vi[e] = bv(c * CW + e, rb[c * CW + e].y);
        }
        const int o = lds_slot(b_col, b_k / CW + c);
        Bsm(b, 0)[o] = vr;
        Bsm(b, 1)[o] = vi;
      }
    } else {
      const int o = lds_slot(b_col, b_k / CW);
      T* pr = reinterpret_cast<T*>(&Bsm(b, 0)[o]) + b_k % CW;
      T* pi = reinterpret_cast<T*>(&Bsm(b, 1)[o]) + b_k % CW;
#pragma unroll
      for (int e = 0; e < BPT; ++e) {
        pr[e] = bv(e, rb[e].x);
        pi[e] = bv(e, rb[e].y);
      }
    }
  };

  // MFMAs of one step from LDS buffer b
  auto compute = [&](int b) {
    VK ar[RBW], ai[RBW], as[RBW];
#pragma unroll
    for (int i = 0; i < RBW; ++i) {
      const int o = lds_slot(16 * (RBW * wr + i) + li, g);
      ar[i] = Asm(b, 0)[o];
      ai[i] = Asm(b, 1)[o];
      as[i] = ar[i] + ai[i];
    }
#pragma unroll
    for (int j = 0; j < CBW; ++j) {
      const int o = lds_slot(16 * (CBW * wc + j) + li, g);
      const VK br = Bsm(b, 0)[o];
      const VK bi = Bsm(b, 1)[o];
      const VK bs = br + bi;
#pragma unroll
      for (int t = 0; t < CW; ++t)
#pragma unroll
        for (int i = 0; i < RBW; ++i) {
          p1[i][j] = nmf<T>::step(ar[i][t], br[t], p1[i][j]);
          p2[i][j] = nmf<T>::step(ai[i][t], bi[t], p2[i][j]);
          p3[i][j] = nmf<T>::step(as[i][t], bs[t], p3[i][j]);
        }
    }
  };
  // Pipeline over the k steps: the loads of step s+1 are issued before the MFMAs of step s
  // and stored into the other LDS buffer after them (one barrier per step).  Steps whose
  // successor is a full step run in a loop with only the 16-byte loads in its body; the
  // last step and a ragged tail step are peeled off.  With PIPE = 2 the full steps keep two
  // steps of loads in flight (register sets alternate, the loop is unrolled by two).
  const int nsteps = (K + KC - 1) / KC;
  const int nvec = vec_steps ? K / KC : 0;  // steps loaded by load_full
  constexpr std::integral_constant<int, 0> set0{};
  if (nvec > 0) load_full(0, set0);
  else load_any(0, set0);
  store(0, set0);
  int st = 0;
  if constexpr (PIPE == 2) {
    constexpr std::integral_constant<int, 1> set1{};
    if (nvec >= 3) {
      // entering each iteration: step st in LDS buffer 0, step st + 1 in flight in set 1
      load_full(KC, set1);
      __syncthreads();
      for (; st + 3 < nvec; st += 2) {
        load_full((st + 2) * KC, set0);
        __builtin_amdgcn_sched_barrier(0);
        compute(0);
        store(1, set1);
        __syncthreads();
        load_full((st + 3) * KC, set1);
        __builtin_amdgcn_sched_barrier(0);
        compute(1);
        store(0, set0);
        __syncthreads();
      }
      compute(0);
      store(1, set1);
      __syncthreads();
      ++st;
    } else {
      __syncthreads();
    }
  } else {
    __syncthreads();
  }
  for (; st + 1 < nvec; ++st) {
    load_full((st + 1) * KC, set0);
    // keep the loads ahead of the MFMAs (the scheduler would sink them to reuse registers)
    __builtin_amdgcn_sched_barrier(0);
    compute(st & 1);
    store((st + 1) & 1, set0);
    __syncthreads();
  }
  for (; st < nsteps; ++st) {
    const bool more = st + 1 < nsteps;
    if (more) load_any((st + 1) * KC, set0);
    compute(st & 1);
    if (more) store((st + 1) & 1, set0);
    __syncthreads();
  }

  // Epilogue through LDS: the output tile is staged column by column (lane: column li of each
  // 16-column block, rows nmf<T>::row(g, q)), then consecutive threads finish consecutive rows
  // of a column, so partial-slice reads and output writes are contiguous runs (coalesced).
  // The operand buffers hold the tile, in column chunks when it does not fit at once.
  constexpr int LDC = ROWS + 1;  // padded column pitch (complex), spreads the lanes over banks
  constexpr int CAP = (int)(sizeof(Ops) / sizeof(cplx<T>)) / LDC;
  constexpr int CPP = CAP >= COLS ? COLS : (CAP >= 32 ? 32 : 16);  // columns per pass
  static_assert(CAP >= 16, "LDS too small for the output tile");
  cplx<T>* Cst = reinterpret_cast<cplx<T>*>(Ops);
  cplx<T>* out = reinterpret_cast<cplx<T>*>(jb.out);
  const cplx<T>* part = reinterpret_cast<const cplx<T>*>(jb.part);
  double2* out64 = reinterpret_cast<double2*>(jb.out64);
  const size_t slice = (size_t)N * M;
  const int dest = jb.dest, nparts = jb.nparts;
  for (int cb = 0; cb < COLS; cb += CPP) {
    __syncthreads();  // previous readers of the LDS block are done
#pragma unroll
    for (int j = 0; j < CBW; ++j) {
      const int cl = 16 * (CBW * wc + j) + li - cb;
      if (cl < 0 || cl >= CPP) continue;
#pragma unroll
      for (int i = 0; i < RBW; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rl = 16 * (RBW * wr + i) + nmf<T>::row(g, q);
          const T a = p1[i][j][q], b2 = p2[i][j][q];
          Cst[cl * LDC + rl] = mk<T>(a - b2, p3[i][j][q] - a - b2);
        }
    }
    __syncthreads();
    if (FINAL && dest == DEST_FINAL) {
      // all outputs of this thread at once: the partial slices are loaded QS at a time for all UPT
      // outputs (up to 32 FP32 / 16 FP64 independent loads in flight), then added in slice order
      constexpr int UPT = CPP * ROWS / 256;
      static_assert(UPT * 256 == CPP * ROWS, "whole outputs per thread");
      constexpr int kLoads = sizeof(T) == 4 ? 32 : 16;
      constexpr int QS = UPT >= kLoads ? 1 : kLoads / UPT;
      size_t at[UPT];
      bool ok[UPT];
      cplx<T> v[UPT];
#pragma unroll
      for (int u = 0; u < UPT; ++u) {
        const int e = tid + 256 * u;
        const int cl = e / ROWS, rl = e - cl * ROWS;
        const int col = col0 + cb + cl, m = m0 + rl;
        ok[u] = col < N && m < M;
        at[u] = ok[u] ? (size_t)col * M + m : 0;  // out-of-range outputs read a valid stand-in
        v[u] = Cst[cl * LDC + rl];
      }
      for (int s0 = 0; s0 < nparts; s0 += QS) {
        cplx<T> pv[UPT][QS];
#pragma unroll
        for (int q = 0; q < QS; ++q)
#pragma unroll
          for (int u = 0; u < UPT; ++u) pv[u][q] = part[(size_t)min(s0 + q, nparts - 1) * slice + at[u]];
#pragma unroll
        for (int q = 0; q < QS; ++q)
          if (s0 + q < nparts)
#pragma unroll
            for (int u = 0; u < UPT; ++u) v[u] = cadd<T>(v[u], pv[u][q]);
      }
#pragma unroll
      for (int u = 0; u < UPT; ++u) {
        if (!ok[u]) continue;
        if (out64) out64[at[u]] = make_double2((double)v[u].x, (double)v[u].y);
        else out[at[u]] = v[u];
      }
      continue;
    }
    for (int e = tid; e < CPP * ROWS; e += 256) {
      const int cl = e / ROWS, rl = e - cl * ROWS;
      const int col = col0 + cb + cl, m = m0 + rl;
      if (col >= N || m >= M) continue;
      if constexpr (DFTG) {
        // output position col of the line, channel m; the last forward pass puts D on the
        // non-canonical bins
        cplx<T> v = Cst[cl * LDC + rl];
        const DftFlip& fl = jobs.dg.flip;
        if (fl.mode == 1 && odd_degree(m, fl.p) && bin_flipped(fl, col, line_u, line_v)) v = mk<T>(-v.x, -v.y);
        out[(size_t)line_off + (size_t)col * lda + m] = v;
        continue;
      }
      size_t base;
      if (ACOL) {
        base = ((size_t)bb * N + col) * M;
      } else if (dest == DEST_GRID) {
        int r, i1, i2, i3;
        cell_coords(jb, col, r, i1, i2, i3);
        const size_t bin = (size_t)i1 + (size_t)jb.N0 * (i2 + (size_t)jb.N1 * i3);
        base = (bin * jb.R + r) * M;
      } else {
        base = (size_t)col * M;
      }
      out[base + m] = Cst[cl * LDC + rl];
    }
  }
}

// The same tile body under two kernel names, so that per-kernel profiles keep the near-field/S2M
// launch apart from the L2T launch even when both use the same tile shape.  WPE: waves per SIMD
// the register allocation must leave room for (3 keeps the MFMA accumulators in ordinary VGPRs
// and three workgroups of four waves per CU; 1 lets the large tiles use the accumulator file).
template <typename T, int ROWS, int COLS, int WR, int KC, int WPE, int PIPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void near_kernel(NearJobs jobs) {
  near_tile<T, ROWS, COLS, WR, KC, PIPE>(jobs);
}
template <typename T, int ROWS, int COLS, int WR, int KC, int WPE, int PIPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void l2t_kernel(NearJobs jobs) {
  near_tile<T, ROWS, COLS, WR, KC, PIPE, false, true>(jobs);
}
template <typename T, int ROWS, int COLS, int WR, int KC, int WPE, int PIPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void m2l_kernel(NearJobs jobs) {
  near_tile<T, ROWS, COLS, WR, KC, PIPE, true>(jobs);
}
template <typename T, int ROWS, int COLS, int WR, int KC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void dft_gemm_kernel(DftGemmJobs jobs) {
  near_tile<T, ROWS, COLS, WR, KC, 1, true, false, DftGemmJobs>(jobs);
}

// y[col][m] = sum_s part[s][col][m] in a fixed order (optionally written as FP64)
template <typename T>
__global__ void near_reduce_kernel(const cplx<T>* __restrict__ part, int ns, size_t len, cplx<T>* __restrict__ y,
                                   double2* __restrict__ y64) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (size_t)gridDim.x * blockDim.x) {
    cplx<T> s = part[i];
    for (int q = 1; q < ns; ++q) s = cadd<T>(s, part[(size_t)q * len + i]);
    if (y64) y64[i] = make_double2((double)s.x, (double)s.y);
    else y[i] = s;
  }
}

// tile shapes: (complex rows, columns, wave rows, complex k per step, waves per SIMD, k steps in
// flight); FP32 steps over 16 complex k (one 16-byte LDS load of 4 floats per operand), FP64 over
// 8 (2 doubles).  The last two were picked per shape by measurement on gfx950 (1280 x 1280
// blocks, 256 columns); the 64 x 128 and 128 x 64 FP64 tiles do not fit three waves per SIMD.
struct NearShape {
  int rows, cols, wr, kc;
};
#define FMBEM_NEAR_SHAPES_F32                                                                   \
  X(0, 64, 128, 2, 16, 3, 1) X(1, 32, 128, 2, 16, 3, 2) X(2, 64, 64, 2, 16, 3, 2)               \
  X(3, 64, 64, 4, 16, 3, 2) X(4, 32, 64, 2, 16, 3, 2) X(5, 16, 128, 1, 16, 3, 1)                \
  X(6, 16, 256, 1, 16, 3, 1) X(7, 128, 64, 4, 16, 3, 1) X(8, 32, 128, 1, 16, 3, 2) X(9, 16, 64, 1, 16, 3, 2)
#define FMBEM_NEAR_SHAPES_F64                                                                   \
  X(0, 64, 128, 2, 8, 1, 1) X(1, 32, 128, 2, 8, 3, 1) X(2, 64, 64, 2, 8, 3, 1)                  \
  X(3, 64, 64, 4, 8, 3, 1) X(4, 32, 64, 2, 8, 3, 2) X(5, 16, 128, 1, 8, 3, 2)                   \
  X(6, 16, 256, 1, 8, 3, 2) X(7, 128, 64, 4, 8, 1, 1) X(8, 32, 128, 1, 8, 3, 1) X(9, 16, 64, 1, 8, 3, 2)
constexpr int kNumShapes = 10;
// M2L products: p rows (121 at n_t = 10) by R columns per bin
#define FMBEM_M2L_SHAPES(KC, W5)                                                                 \
  X(0, 64, 64, 4, KC, 3, 1) X(1, 32, 64, 2, KC, 3, 1) X(2, 64, 32, 2, KC, 3, 1) X(3, 32, 32, 2, KC, 3, 1) \
  X(4, 16, 64, 1, KC, 3, 1) X(5, 128, 64, 4, KC, W5, 1) X(6, 32, 64, 2, KC, 3, 2) X(7, 64, 32, 2, KC, 3, 2)     \
  X(8, 64, 64, 4, KC, 2, 2) X(9, 64, 64, 2, KC, 2, 2)
constexpr int kNumM2lShapes = 10;
template <typename T> constexpr int shape_kc() { return sizeof(T) == 4 ? 16 : 8; }
template <typename T> constexpr int m2l_w5() { return sizeof(T) == 4 ? 2 : 1; }

template <typename T>
static NearShape shape_of(int kind, int v) {
#define X(i, r, c, w, k, wpe, pipe) \
  case i: return NearShape{r, c, w, k};
  if (kind == 2) {
    switch (v) { FMBEM_M2L_SHAPES(shape_kc<T>(), m2l_w5<T>()) }
    return NearShape{64, 64, 4, shape_kc<T>()};
  }
  if constexpr (sizeof(T) == 4) {
    switch (v) { FMBEM_NEAR_SHAPES_F32 }
  } else {
    switch (v) { FMBEM_NEAR_SHAPES_F64 }
  }
#undef X
  return NearShape{64, 128, 2, shape_kc<T>()};
}

template <typename T>
int near_num_shapes(int kind) {
  return kind == 2 ? kNumM2lShapes : kNumShapes;
}

template <typename T>
static void launch_shape(int v, int kind, unsigned blocks, const NearJobs& jobs, hipStream_t s) {
  if (kind == 2) {
    switch (v) {
#define X(i, r, c, w, k, wpe, pipe) \
  case i: hipLaunchKernelGGL((m2l_kernel<T, r, c, w, k, wpe, pipe>), dim3(blocks), dim3(256), 0, s, jobs); break;
      FMBEM_M2L_SHAPES(shape_kc<T>(), m2l_w5<T>())
#undef X
    }
    return;
  }
#define X(i, r, c, w, k, wpe, pipe)                                                                             \
  case i:                                                                                                      \
    if (kind == 1) hipLaunchKernelGGL((l2t_kernel<T, r, c, w, k, wpe, pipe>), dim3(blocks), dim3(256), 0, s, jobs); \
    else hipLaunchKernelGGL((near_kernel<T, r, c, w, k, wpe, pipe>), dim3(blocks), dim3(256), 0, s, jobs);          \
    break;
  if constexpr (sizeof(T) == 4) {
    switch (v) { FMBEM_NEAR_SHAPES_F32 }
  } else {
    switch (v) { FMBEM_NEAR_SHAPES_F64 }
  }
#undef X
}

template <typename T>
static long long job_tiles(const NearJob& j, const NearShape& sh) {
  return (long long)j.batch * ((j.M + sh.rows - 1) / sh.rows) * ((j.N + sh.cols - 1) / sh.cols);
}

// Relative throughput of each near-field shape on a large problem (1280 x 1280 blocks, 256
// columns; measured on gfx950), the prior of the default choice.
static const double kPriorF32[kNumShapes] = {0.75, 0.94, 1.0, 0.99, 0.93, 0.66, 0.36, 0.66, 0.94, 0.72};
static const double kPriorF64[kNumShapes] = {0.50, 0.97, 1.0, 1.0, 0.96, 0.89, 0.54, 0.50, 0.96, 0.90};

// default shape (untuned signatures): measured prior x fill of the last round of workgroups
template <typename T>
static int near_default_shape(const std::vector<NearJob>& jobs, int kind) {
  int best = 0;
  double best_score = -1.0;
  for (int v = 0; v < near_num_shapes<T>(kind); ++v) {
    const NearShape sh = shape_of<T>(kind, v);
    long long wg = 0;
    for (const NearJob& j : jobs) wg += job_tiles<T>(j, sh);
    const long long rounds = (wg + 255) / 256;
    const double fill = (double)wg / (double)(rounds * 256);
    const double prior = kind == 2 ? 1.0 : (sizeof(T) == 4 ? kPriorF32[v] : kPriorF64[v]);
    const double score = prior * fill;
    if (score > best_score) {
      best_score = score;
      best = v;
    }
  }
  return best;
}

template <typename T>
hipError_t near_launch(const std::vector<NearJob>& list, hipStream_t s, int shape, int kind) {
  if (list.empty()) return hipSuccess;
  // DEST_FINAL jobs need the L2T kernel's epilogue, and only those go to it
  for (const NearJob& j : list)
    if ((j.dest == DEST_FINAL) != (kind == 1)) return hipErrorInvalidValue;
  if (shape < 0 || shape >= near_num_shapes<T>(kind)) shape = near_default_shape<T>(list, kind);
  const NearShape sh = shape_of<T>(kind, shape);
  for (size_t first = 0; first < list.size(); first += kMaxJobs) {
    NearJobs jobs;
    jobs.count = (int)std::min<size_t>(kMaxJobs, list.size() - first);
    long long tiles = 0;
    for (int j = 0; j < jobs.count; ++j) {
      jobs.job[j] = list[first + j];
      jobs.job[j].tile0 = (int)tiles;
      tiles += job_tiles<T>(jobs.job[j], sh);
    }
    if (tiles == 0) continue;
    if (tiles > INT32_MAX) return hipErrorInvalidValue;
    jobs.total = (int)tiles;
    launch_shape<T>(shape, kind, (unsigned)tiles, jobs, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// DFT passes: the tile width is the smallest of 32 / 64 / 128 output columns that holds every
// output of the pass (one column tile per line, so the pass can run in place); rows = channels
template <typename T>
hipError_t dft_gemm_launch(const NearJob& job, const DftGemm& dg, hipStream_t s) {
  if (job.N > kDftGemmMaxOut || job.batch < 1 || job.M < 1 || job.K < 1 || !job.A || !job.src) return hipErrorInvalidValue;
  constexpr int kc = shape_kc<T>();
  DftGemmJobs jl;
  jl.count = 1;
  jl.job[0] = job;
  jl.job[0].tile0 = 0;
  jl.dg = dg;
  const int rows = job.N <= 64 ? 64 : 32;
  const long long tiles = (long long)job.batch * ((job.M + rows - 1) / rows);
  if (tiles > INT32_MAX) return hipErrorInvalidValue;
  jl.total = (int)tiles;
  if (job.N <= 32)
    hipLaunchKernelGGL((dft_gemm_kernel<T, 64, 32, 2, kc>), dim3((unsigned)tiles), dim3(256), 0, s, jl);
  else if (job.N <= 64)
    hipLaunchKernelGGL((dft_gemm_kernel<T, 64, 64, 4, kc>), dim3((unsigned)tiles), dim3(256), 0, s, jl);
  else
    hipLaunchKernelGGL((dft_gemm_kernel<T, 32, 128, 1, kc>), dim3((unsigned)tiles), dim3(256), 0, s, jl);
  return hipGetLastError();
}

template <typename T>
hipError_t near_reduce_launch(const void* part, int ns, size_t len, void* y, void* y64, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<size_t>((len + 255) / 256, 8192);
  hipLaunchKernelGGL(near_reduce_kernel<T>, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const cplx<T>*>(part),
                     ns, len, reinterpret_cast<cplx<T>*>(y), reinterpret_cast<double2*>(y64));
  return hipGetLastError();
}

template hipError_t dft_gemm_launch<double>(const NearJob&, const DftGemm&, hipStream_t);
template hipError_t dft_gemm_launch<float>(const NearJob&, const DftGemm&, hipStream_t);
template hipError_t near_launch<double>(const std::vector<NearJob>&, hipStream_t, int, int);
template hipError_t near_launch<float>(const std::vector<NearJob>&, hipStream_t, int, int);
template int near_num_shapes<double>(int);
template int near_num_shapes<float>(int);
template hipError_t near_reduce_launch<double>(const void*, int, size_t, void*, void*, hipStream_t);
template hipError_t near_reduce_launch<float>(const void*, int, size_t, void*, void*, hipStream_t);

}  // namespace fmbem
