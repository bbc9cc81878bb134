// Internal declarations of the fmbem HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "fmbem.h"

namespace fmbem {

// ---------------------------------------------------------------------------
// complex helpers: interleaved (re, im) as HIP vector types
// ---------------------------------------------------------------------------
template <typename T> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };
template <typename T> using cplx = typename cplx_t<T>::type;

template <typename T>
__host__ __device__ inline cplx<T> mk(T re, T im) { cplx<T> c; c.x = re; c.y = im; return c; }
template <typename T>
__host__ __device__ inline cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__host__ __device__ inline cplx<T> csub(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__host__ __device__ inline cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__host__ __device__ inline cplx<T> cconj(cplx<T> a) { return mk<T>(a.x, -a.y); }
template <typename T>
__host__ __device__ inline cplx<T> cscale(cplx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// a += b * c
template <typename T>
__host__ __device__ inline void cfma(cplx<T>& a, cplx<T> b, cplx<T> c) {
  a.x += b.x * c.x - b.y * c.y;
  a.y += b.x * c.y + b.y * c.x;
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
constexpr int kMaxNear = 343;   // (2*3+1)^3 near offsets at near radius 3
constexpr int kDftGemmMaxOut = 128;  // widest output count of a DFT pass as a GEMM (one tile width)

// Gauss-Legendre rules on [0, 1] (nodes t, weights w) for q = 4, 8, 16 points,
// stored at offsets 0, 4 and 12 (28 entries)
struct QuadTab {
  double t[28];
  double w[28];
};

// Multilevel near field (FMPBEM2, Sec. 3.3): launch tables of the block-sparse products.
// Output rows [out_row, out_row + rows) of a stage's output buffer (rows <= 64) receive the sum
// of the target's tasks; a task multiplies the operator A (rows x ks, row-major with row stride
// lda, at ops + a_off) into source rows [src_row, src_row + ks) of buffer sel & 3, taken at the
// column of cell c - d for output cell c (d = the cell shift sel >> 2, encoded as
// (d0 + 1) + 3 (d1 + 1) + 9 (d2 + 1); zero outside the lattice).  Buffers ([rows][R C]): 0 the
// input in tree order, 1 moments, 2 locals, 3 the output in tree order.
struct MlTarget {
  int out_row, rows, t0, t1;
};
struct MlTask {
  long long a_off;
  int lda, ks, src_row, sel;
};
struct MlStage {
  const MlTarget* tg;  // device, n_tg targets
  const MlTask* tk;    // device (all tasks of the plan)
  int n_tg;
  int out, accum;      // output buffer; 1: add to it
  int max_rows;        // largest target
  // split > 1: each target's tasks are divided over `split` workgroups that write the partial
  // buffer `part` (slot s at rows s nrows + out_row - row0); the slots are then added in slot order
  // into rows [row0, row0 + nrows) of buffer `dest` (added to it when dest_accum)
  int split = 1, dest = 0, dest_accum = 0, row0 = 0, nrows = 0, part = 5;
};
struct MlData {
  int levels = 0, order = 0, p = 0;
  int rows = 0;                      // expansion rows of levels 1..L (p per box)
  int* pos = nullptr;                // device [n]: tree position of every element
  int* perm = nullptr;               // device [n]: element at every tree position
  void* ops[2] = {nullptr, nullptr}; // operator pool FP64 / FP32 (P2M, L2P, M2M, L2L, M2L, P2P)
  size_t ops_elems = 0;
  std::vector<MlStage> stages;       // P2M, M2M per level, M2L, L2L per level, L2P (added to the P2P)
  MlStage p2p{};                     // the exact leaf blocks, from the input alone (written first)
  // S2M of the cell-level far field from the input in tree order: V0 with its columns in tree
  // order at ops + oS, products over chunks of the elements into partial sums (buffer 4), summed
  // in chunk order into the padded grid
  MlStage s2m{};
  long long oS = 0;
  int s2m_chunks = 0;
  size_t part_rows = 0;              // rows of the partial buffer of the split M2L (split x nrows)
  size_t p2p_part_rows = 0;          // rows of the partial buffer of the split P2P stage
  int max_tasks = 0;                 // longest task list of one launched target (any stage)
  int boxes = 0, leaves = 0;
  long long m2l_pairs = 0, p2p_pairs = 0, p2p_entries = 0;
  double macs_per_rhs = 0.0;         // complex multiply-adds of one application per RHS (cells inside)
};
// exact entries of one P2P block: rows = tree positions [te0, te0 + nt), columns [se0, se0 + ns)
// of S_d (shift index sd as in MlTask), row-major at ops + off
struct P2pBlock {
  long long off;
  int te0, nt, se0, ns, sd;
};

struct Plan {
  int device = 0;
  int n = 0;                 // triangles (DOFs) per cell
  int grid[3] = {1, 1, 1};
  int C = 1;
  double pitch[3] = {1, 1, 1};
  double k = 1.0;
  int order = 0, p = 1, p2 = 1;  // p = (nt+1)^2, p2 = (2nt+1)^2
  int formulation = 0;
  double alpha_re = 0, alpha_im = 0;
  int near_radius[3] = {1, 1, 1};
  int fft[3] = {1, 1, 1};
  int B = 1;
  uint32_t precisions = 1;
  double scale = 1.0;        // diagonal scaling s: V0 rows / s^n, U0 cols / s^n, Lambda * s^(n+n')
  int n_near = 0, n_far = 0;
  std::vector<int> near_off; // [n_near][3]
  // device arrays (owned)
  QuadTab quad{};            // element quadrature rules (see QuadTab)
  double* geom = nullptr;    // [n][18]: a(3) b(3) c(3) centroid(3) normal(3) longest, area, pad
  int* d_near = nullptr;     // [n_near][3]
  void* S[2] = {nullptr, nullptr};    // [n_near][n][n] complex, row-major
  void* V0[2] = {nullptr, nullptr};   // [p][n] complex, row-major, scaled
  void* U0[2] = {nullptr, nullptr};   // [n][p] complex, row-major, scaled
  void* Lam[2] = {nullptr, nullptr};  // [Bc][p(col)][ldp] complex: per canonical bin, column-major, scaled, /B
  // DFT matrices of the grid axes (GEMM schedule), per precision: forward of axis a at [a]
  // ([N_a][M_a], w^(k j) with w = e^(-2 pi i / N_a)), inverse at [3 + a] ([M_a][N_a], conjugate
  // kernel); only for 1 < N_a <= kDftGemmMaxOut, else nullptr
  void* dftF[2][6] = {};
  int tile_forced[3] = {-1, -1, -1};  // tile shapes forced by the plan descriptor (-1: tuned)
  int dft_forced = -1;       // DFT schedule forced by the plan descriptor (0 axes, 1 fused, 2 GEMM, 3 fused
                             // on the matrix cores), -1: tuned
  // half-space: image term R_p G(x, y^) with y^ mirrored in z = zg.  half: the incident fields
  // and the field evaluation carry the image; fold (plane parallel to every periodic axis,
  // grid[2] == 1): the image blocks are added to this plan's S and Lambda; otherwise (periodic
  // along z) the image part, block Hankel along z, is the sub-plan img applied to the input
  // reversed along z (Sec. 2.3, Sec. 3.5: the column permutation P)
  bool half = false, fold = false;
  double zg = 0.0, rp_re = 0.0, rp_im = 0.0;
  bool img_near = false;     // fold: the image blocks of the near offsets are near blocks too
  int n_far_img = 0;         // fold: image offsets applied through the multipole chain
  struct Plan* img = nullptr;        // image sub-plan (owned), periodic along z
  const struct Plan* parent = nullptr;  // set in an image sub-plan: geometry, V0, U0, DFT matrices shared
  // the canonical-bin pairing Lambda(-w) = D Lambda(w) D holds (off in the half-space, whose
  // image part pairs differently): when off every bin is stored and the DFT applies no D
  bool paired = true;
  // exact periodic BEM (comparison method): Lambda holds the n x n exact blocks per bin, V0 = U0 = I,
  // no near blocks, p = n
  bool exact = false;
  // multilevel near field (FMPBEM2): set => no dense near blocks (n_near = 0), the near offsets
  // of radius 1 are applied by the multilevel FMM after the far field
  std::shared_ptr<MlData> ml;
  int flip_p() const { return paired ? p : 0; }
  // Lambda of bin -w is D Lambda(w) D, D = diag((-1)^n) (reciprocity of the translations), so only
  // canonical bins (linear index <= that of the partner bin -w) are stored.
  int Bc = 0;                // canonical bins
  int* d_canon = nullptr;    // [B] canonical slot of every bin
  int* d_pairs = nullptr;    // [Bc][2] (bin, partner bin or -1 when the bin is its own partner)
  size_t resident = 0;
  std::vector<void*> allocations;
  // stage profiling (HIP events on the caller's stream)
  struct Prof {
    uint32_t mask = 0;                                // recorded stages (bit per stage)
    int period = 1;                                   // record every period-th application
    long long calls = 0;                              // applications since profiling started
    bool active = false;                              // the current application is recorded
    std::vector<hipEvent_t> pool;                     // free events
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;  // (stage, start, stop)
    double ms[FMBEM_N_STAGES] = {0};
    long long count[FMBEM_N_STAGES] = {0};
  };
  mutable Prof prof;
  // second stream (default priority) on which the far-field chain of a single-plan apply runs
  // while the near field runs on the caller's stream; fork/join events; the lock keeps the
  // event pair consistent between concurrent applications
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::unique_ptr<std::mutex> aux_mu{new std::mutex};
};

inline fmbem_status to_status(hipError_t e) {
  if (e == hipSuccess) return FMBEM_OK;
  if (e == hipErrorOutOfMemory) return FMBEM_ERR_OUT_OF_MEMORY;
  return FMBEM_ERR_DEVICE;
}

// record the start / end of a stage when that stage is being profiled (returns the start event);
// counted = false: the interval adds its time to the stage but not to its count of applications
constexpr int kProfUncounted = 0x100;
hipEvent_t prof_begin(const Plan& P, int stage, hipStream_t s);
void prof_end(const Plan& P, int stage, hipEvent_t start, hipStream_t s, bool counted = true);

size_t matvec_workspace_bytes_per_rhs(const Plan& P, int precision);

// multilevel near field (multilevel.hip): tree and operators (plan build), workspace, application
// (y (+)= the near field of x; y64: complex128 output of an FP32 application).  Parts (bit mask):
// ml_prepare 1 = the input into tree order, 2 = the S2M from it; ml_apply 1 = the products into
// the tree-ordered output, 2 = that output added to (or written into) y
bool ml_cell_fits(const std::vector<double>& geo, int n, const double pitch[3], int L);
hipError_t ml_build(Plan& P, const std::vector<double>& geo, hipStream_t s);
size_t ml_workspace_bytes_per_rhs(const Plan& P, int precision);
template <typename T>
hipError_t ml_prepare(const Plan& P, int R, const void* x, void* ws, void* grid, hipStream_t s, int parts = 3);
template <typename T>
hipError_t ml_apply(const Plan& P, int R, void* y, void* y64, void* ws, bool accum, hipStream_t s, int parts = 3);
// plan.hip helpers used by the multilevel build
hipError_t plan_alloc(Plan& P, void** ptr, size_t bytes);
void gauss_legendre_host(int q, std::vector<double>& x, std::vector<double>& w);
void theta_table(int L, const std::vector<double>& x, std::vector<double>& tab);
hipError_t cast_launch(const double2* a, float2* b, size_t n, hipStream_t s);
// leaf P2M (columns of ops + oV, row stride n) and L2P (rows of ops + oU, row stride p) about the
// leaf centre of every element (cen, host [n][3]) with the column / row scaling isig (host),
// and the exact entries of the P2P blocks
hipError_t ml_assemble_launch(const Plan& P, int nt, const std::vector<double>& cen, const std::vector<double>& isig,
                              const std::vector<P2pBlock>& blocks, long long entries, double2* ops, long long oV,
                              long long oU, hipStream_t s);

// stream-ordered operator application (all arguments validated by the caller);
// y64 (FP32 only, optional): write the result as complex128 there instead of y
// tune: autotune the tile shapes of a new problem signature (blocks the host once per
// signature); otherwise a shape tuned earlier for the same signature, or the default.
hipError_t matvec_launch(const Plan& P, int precision, int R, const void* x, void* y, void* ws,
                         hipStream_t s, void* y64 = nullptr, bool tune = true);

// one operator application of a group (see matvec_group)
struct GroupApply {
  const Plan* P;
  int R;
  const void* x;   // [R][C][n] in the application's precision
  void* y;         // [R][C][n] in that precision (unused when y64 is set)
  void* ws;        // R * matvec_workspace_bytes_per_rhs(P, precision), 256-byte aligned
  void* y64;       // FP32 only, optional: complex128 output
};
// Applications of several plans in one precision, their near-field + S2M and L2T GEMMs in
// shared grouped launches; stream-ordered.  tune: autotune the combined tile shape.
hipError_t matvec_group(int precision, const std::vector<GroupApply>& g, hipStream_t s, bool tune);

// ---------------------------------------------------------------------------
// kernels shared between translation units
// ---------------------------------------------------------------------------
constexpr int kMaxSeg = 32;        // near offsets per plan (3-D lattices with near radius 1 need 27)
constexpr int kMaxGridDim = 4096;  // lattice cells per axis
constexpr int kMaxJobs = 34;       // GEMM jobs per grouped launch (larger groups are split)

// Grouped complex GEMM jobs on the near-field kernel (near.hip): out = A B with A complex
// [M][K] row-major (row stride lda) and N columns; column j is (RHS r, cell c) =
// (j / C, j % C) of the job's lattice.  Its B column is x_{r, c - d} (SRC_X: src holds
// [R][C][K], zero outside the lattice) or the padded-grid entry of cell c (SRC_GRID: src
// holds [bin][R][K]).  A batched job (SRC_BATCH, M2L kernel) is batch independent GEMMs:
// A_b column-major [K][lda] at A + slot(b) K lda (slot(b) = amap[b], or b without a map),
// B_b columns at src + (b N + j) K, output
// column j of product b at out + (b N + j) M.
enum NearSrc : int { SRC_X = 0, SRC_GRID = 1, SRC_BATCH = 2 };
enum NearDest : int {
  DEST_SLICE = 0,  // out [N][M] column-major
  DEST_GRID = 1,   // out padded grid [bin][R][M]
  DEST_FINAL = 2   // out [N][M] = acc + sum of nparts slices of part (same layout); FP64 to out64 if set
};
struct NearJob {
  const void* A;
  void* out;
  const void* src;
  const void* part;
  void* out64;
  const int* amap;           // SRC_BATCH: A slot of every product (nullptr: slot = product index)
  int M, K, N;
  int lda;                   // A row stride (row-major) or column stride (SRC_BATCH)
  int batch;                 // products in a SRC_BATCH job (1 otherwise)
  int tile0;                 // first logical workgroup (set by near_launch)
  int C, R;                  // cells and RHS of the job's lattice
  short M0, M1, M2, N0, N1;  // lattice and padded-grid dims
  short d0, d1, d2;          // cell offset of the B columns (SRC_X)
  short nparts;
  char src_kind, dest;
};
struct NearJobs {
  int count;
  int total;  // workgroups
  NearJob job[kMaxJobs];
};
inline NearJob near_job(const Plan& P, int R, const void* A, void* out, int M, int K, const void* src, int src_kind,
                        int dest) {
  NearJob j{};
  j.A = A;
  j.out = out;
  j.src = src;
  j.M = M;
  j.K = K;
  j.lda = K;
  j.batch = 1;
  j.N = R * P.C;
  j.C = P.C;
  j.R = R;
  j.M0 = (short)P.grid[0];
  j.M1 = (short)P.grid[1];
  j.M2 = (short)P.grid[2];
  j.N0 = (short)P.fft[0];
  j.N1 = (short)P.fft[1];
  j.src_kind = (char)src_kind;
  j.dest = (char)dest;
  return j;
}

// Launch a list of jobs (split into launches of at most kMaxJobs).  shape < 0: default tile
// shape; else one of near_num_shapes<T>(kind) shapes.  kind 0 launches the tile body as
// near_kernel (near field + S2M), 1 as l2t_kernel (L2T), 2 as m2l_kernel (SRC_BATCH jobs,
// column-major A).
template <typename T>
hipError_t near_launch(const std::vector<NearJob>& jobs, hipStream_t s, int shape = -1, int kind = 0);
template <typename T>
int near_num_shapes(int kind);
// y = sum of ns partial slices (FP64 to y64 when set)
template <typename T>
hipError_t near_reduce_launch(const void* part, int ns, size_t len, void* y, void* y64, hipStream_t s);

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

// -c mod n for 0 <= c < n, without a division
__device__ inline int neg_mod(int c, int n) { return c == 0 ? 0 : n - c; }

__device__ inline bool bin_flipped(const DftFlip& f, int pos, int u, int v) {
  int c[3];
  const int b = f.axis == 0 ? 1 : 0, d = f.axis == 2 ? 1 : 2;
  c[f.axis] = pos;
  c[b] = u;
  c[d] = v;
  const long long L = c[0] + (long long)f.N[0] * (c[1] + (long long)f.N[1] * c[2]);
  const long long Lp = neg_mod(c[0], f.N[0]) +
                       (long long)f.N[0] * (neg_mod(c[1], f.N[1]) + (long long)f.N[1] * neg_mod(c[2], f.N[2]));
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

// One axis pass of the grid DFT as a batched MFMA GEMM on the tile body of near.hip, in place:
// for every line (u, v) of the pass, the transposed form out_line^T = X_line^T F^T with rows =
// channels (contiguous), k = input positions along the axis (element stride lda), columns =
// output positions.  The job is SRC_BATCH-like: A = the grid buffer, src = F [Mout][Min] (the
// column of output k is row k of F, contiguous), out = the grid buffer, batch = lines.  In
// place is safe because one workgroup holds every output column of its channels (N <= the tile
// width, checked by the launcher) and reads all of its inputs before it writes.
struct DftGemm {
  long long su, sv;  // element offsets of line indices u (< U) and v
  int U;
  DftFlip flip;      // mode 1: negate the flipped outputs, 2: negate the flipped inputs
};
struct DftGemmJobs {  // one job, with the list interface of the tile body
  int count;
  int total;
  NearJob job[1];
  DftGemm dg;
};
template <typename T>
hipError_t dft_gemm_launch(const NearJob& job, const DftGemm& dg, hipStream_t s);

// flip_p > 0: the channels are [..][p] multipole coefficients and the spectrum of every
// non-canonical bin carries the factor D = diag((-1)^n): applied to the forward output and
// removed from the inverse input (then Lambda of the canonical partner serves that bin).
// schedule: 0 separate axis passes, 1 the fused two-axis kernel where it applies (else the
// passes), 2 axis passes as MFMA GEMMs with the DFT matrices fmat (forward of axis a at
// fmat[a], inverse at fmat[3 + a]) where they apply (else the passes), 3 both axes on the
// matrix cores, 4 both axes as mixed-radix FFTs in one launch, -1 the built-in rule (the FFT
// where it applies; else fused for at most 256 channels, the GEMM passes where they apply).
template <typename T>
hipError_t grid_dft_launch(void* buf, int channels, const int M[3], const int N[3], bool inverse,
                           bool pruned, hipStream_t s, int flip_p = 0, int schedule = -1,
                           const void* const* fmat = nullptr);
// whether the GEMM schedule applies (matrices present for every transformed axis, pruned, every
// pass has at most kDftGemmMaxOut outputs and int-sized strides)
template <typename T>
bool dft_gemm_applies(int channels, const int M[3], const int N[3], bool pruned, const void* const* fmat);
template <typename T>
bool dft_mfma_applies(int channels, const int M[3], const int N[3], bool pruned, const void* const* fmat);
// whether the fused two-axis kernel applies (N3 = 1, N1 > 1, pruned, one channel fits its LDS)
template <typename T>
bool dft_fused_applies(int channels, const int M[3], const int N[3], bool pruned);
// whether the fused two-axis FFT applies (N3 = 1, pruned, the slab of one channel fits the LDS)
template <typename T>
bool dft_fft_applies(int channels, const int M[3], const int N[3], bool pruned);
// one grid transform of the FFT schedule (pruned forward / cropped inverse, as grid_dft_launch)
struct FftTransform {
  void* buf;
  int channels;
  int M[3], N[3];
  int flip_p;
};
// the FFT schedule of several grids, grouped into as few launches as possible (each grid must
// satisfy dft_fft_applies); the result of each equals that of its own launch bit for bit
template <typename T>
hipError_t fft2_group_launch(const std::vector<FftTransform>& tr, bool inverse, hipStream_t s);

// column stride (complex elements) of the per-bin column-major Lambda blocks
int lambda_ld(int p);
// per-bin M2L GEMV, in place in buf [B][R][p]; one workgroup per canonical bin applies its Lambda
// to the R vectors of the bin and of its partner
template <typename T>
hipError_t m2l_launch(const void* Lam, const int* pairs, int Bc, void* buf, int R, int p, hipStream_t s);
// one plan's GEMV product (in place in buf) within a grouped launch
struct M2lProduct {
  const void* Lam;
  const int* pairs;
  int Bc;
  void* buf;
  int R, p;
};
// the GEMV products of several plans in as few launches as their orders allow (one per kernel form);
// each result equals that of its own launch bit for bit
template <typename T>
hipError_t m2l_group_launch(const std::vector<M2lProduct>& v, hipStream_t s);
// right-hand-side count from which the M2L runs as a batched MFMA GEMM into a second buffer (the GEMV
// streams Lambda once per 4 vectors of a bin pair: at 5 or more right-hand sides the GEMM, which
// reads it once per bin, is faster; measured on 16 x 16 and 40 x 8 lattices at n_t = 10)
constexpr int kM2lGemmRhs = 5;

}  // namespace fmbem
