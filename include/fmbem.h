/*
 * fmbem.h - C ABI of the MI355X (gfx950) fast multipole periodic BEM library.
 *
 * The library applies and solves the single-level fast multipole periodic
 * boundary element operator of Jelich, Zhao, Chen & Marburg (arXiv 2201.12050):
 * a unit-cell surface mesh of flat constant triangles is replicated on an
 * M1 x M2 x M3 axis-aligned lattice, each cell is one FMM box, and the rigid-body
 * Burton-Miller (or CBIE) collocation operator is approximated by
 *
 *     A  ~  S + U K V          (Sec. 3.1, eq. (SingleLevelFMM); Sec. 3.2, eq. (2dPeriodicFMM))
 *
 * with S the banded multilevel block-Toeplitz near field, U = diag(U0) and
 * V = diag(V0) the per-cell L2P and P2M operators and K the multilevel
 * block-Toeplitz M2L operator, applied through its circulant embedding as
 * U F^-1 Lambda F V (Sec. 2.4, eq. (diagonalized); Sec. 3.5, eq. (FMPBEMsystem)).
 *
 * Conventions for every entry point:
 *  - No C++ exception crosses the ABI; every call returns fmbem_status.
 *  - Argument errors are detected before any device work is enqueued; on an
 *    error nothing is written.
 *  - Complex numbers are interleaved (re, im) pairs: complex128 (two doubles)
 *    or complex64 (two floats), matching torch.complex128 / torch.complex64.
 *  - Vector layout [n_rhs][n_cells][n_dof_cell]: cell c = i1 + M1*(i2 + M2*i3),
 *    DOF within a cell = triangle index of the unit-cell mesh.
 *  - "device" pointers are HIP device memory on the device that was current
 *    when the plan was created; "host" pointers are ordinary host memory.
 *  - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *    Stream-ordered calls return before the work completes.
 */
#ifndef FMBEM_H
#define FMBEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FMBEM_OK = 0,
  FMBEM_ERR_INVALID_ARG = 1,   /* bad pointer, size, mesh or descriptor field */
  FMBEM_ERR_UNSUPPORTED = 2,   /* valid request the library does not implement */
  FMBEM_ERR_OUT_OF_MEMORY = 3, /* a device allocation failed; nothing leaked */
  FMBEM_ERR_DEVICE = 4,        /* a HIP call failed (no device, launch failure) */
  FMBEM_ERR_NOT_CONVERGED = 5, /* solve stopped at its iteration limit; x = last iterate */
  FMBEM_ERR_WORKSPACE = 6,     /* caller workspace smaller than fmbem_plan_info says */
  FMBEM_ERR_ADMISSION = 7      /* serving engine: the request can never fit the byte budget */
} fmbem_status;

typedef enum { FMBEM_FP64 = 0, FMBEM_FP32 = 1 } fmbem_precision;
typedef enum { FMBEM_BURTON_MILLER = 0, FMBEM_CBIE = 1 } fmbem_formulation;

typedef struct fmbem_plan_s* fmbem_plan;
typedef struct fmbem_engine_s* fmbem_engine;
typedef struct fmbem_solver_s* fmbem_solver;

/* Unit-cell mesh in cell-local coordinates: the cell centre (= expansion centre
 * of its FMM box, Sec. 3.2) is the origin.  Copied during fmbem_plan_create. */
typedef struct {
  int32_t n_vertices;
  const double* vertices;     /* host [n_vertices][3], metres */
  int32_t n_triangles;
  const int32_t* triangles;   /* host [n_triangles][3], 0-based; (v1-v0)x(v2-v0) points
                                 out of the fluid, into the scatterer (Sec. 2.1) */
} fmbem_cell_mesh;

typedef struct {
  int32_t grid[3];            /* M1, M2, M3 >= 1 (each <= 4096, else FMBEM_ERR_UNSUPPORTED) */
  double pitch[3];            /* lattice spacing per axis (m), > 0 */
  double k;                   /* wavenumber k = 2 pi f / c > 0 (1/m), Sec. 2.1 */
  int32_t order;              /* truncation number n_t in [0, 20]; p = (n_t+1)^2 (Sec. 3.1) */
  int32_t formulation;        /* fmbem_formulation */
  double alpha_re, alpha_im;  /* Burton-Miller coupling; both NaN => -i/k (Sec. 2.1) */
  int32_t near_radius[3];     /* near field: |d_a| <= near_radius_a cells (0 => 1) */
  int32_t fft_shape[3];       /* 0 => 2 M_a on the axes of a lattice with M3 = 1 (even lengths for the
                                 FFT schedule), 2 M_a - 1 (the smallest exact embedding) otherwise,
                                 1 where M_a = 1; else >= 2 M_a - 1 (<= 8192) */
  uint32_t precisions;        /* bitmask (1<<FMBEM_FP64) | (1<<FMBEM_FP32) of resident copies;
                                 0 => FP64 only */
  int32_t dft_schedule;       /* FMBEM_DFT_*: how the grid DFT (Sec. 2.4) runs; AUTO measures the
                                 applicable schedules on first use of each problem signature; a
                                 forced schedule that does not apply falls back to AXES */
  /* Half-space (Sec. 2.1, eq. (green3dHalf); Sec. 2.3; Sec. 3.4): halfspace = 1 adds to every
   * interaction the image term R_p G(x, y^), y^ the mirror image of y in the plane
   * z = plane_z, applied as image near blocks and an image multipole chain (Appendix A,
   * eq. (greenFMMhalfspace)); the incident fields and fmbem_field get their images too.  With
   * grid[2] == 1 (the plane parallel to every periodic direction) the image part is block
   * Toeplitz and shares the plan's operator; with grid[2] > 1 it is block Hankel along z and
   * is applied as a second operator to the input reversed along z (a second apply per
   * fmbem_matvec, more workspace).  No layer of cells may cross the plane (touching is allowed;
   * else FMBEM_ERR_INVALID_ARG).  An image block is near when its in-plane offset is a near
   * offset and its z offset |s pitch[2] - 2 plane_z| < (near_radius[2] + 1) pitch[2], s = the
   * sum of the target's and the source's z indices.  halfspace = 0: full space (the other
   * three fields are ignored). */
  int32_t halfspace;
  double plane_z;
  double reflection_re, reflection_im;  /* R_p */
  /* Tile shape of the grouped MFMA launches of this plan, [near field + S2M, L2T, M2L GEMM]:
   * 0 => autotuned (measured on first use of each launch signature); v in
   * 1..FMBEM_TILE_SHAPES => shape v - 1 of that launch's list, so that every shape can be
   * checked.  The M2L GEMM shape holds wherever the plan is applied; the near-field and L2T
   * shapes hold for the plan's own applies (fmbem_matvec, fmbem_solve, fmbem_solver_*), while
   * batched solves and the engine tune the launches they share between plans.  Outside
   * 0..FMBEM_TILE_SHAPES => FMBEM_ERR_INVALID_ARG. */
  int32_t tile_shape[3];
  /* exact = 1: the exact periodic BEM operator (PBEM, Sec. 2.2 eq. (toeplitzBEM), Sec. 2.4
   * eqs. (blockDiagonal), (diagonalized)) instead of the fast multipole one: every block S_d of
   * the lattice (|d_a| <= M_a - 1) is integrated with the element quadrature, the first block
   * column of its circulant embedding is transformed over the grid, and each bin holds an n x n
   * block (no truncation: the matrix is the dense collocation matrix, applied in
   * O(B n^2) per right-hand side).  The same operator application and solvers run on it (the
   * expansion space is the element space: P2M and L2P are identities).  order and near_radius
   * are ignored; the half-space is not supported (FMBEM_ERR_UNSUPPORTED).  The paper's
   * comparison method; the plan stores B n^2 complex values per precision.  0 => FMPBEM. */
  int32_t exact;
  /* near_levels = L >= 1: the multilevel near field of FMPBEM2 (Sec. 3.3).  The lattice box of
   * the unit cell (edge = pitch per axis, centred on the cell centre) is halved L times along
   * every axis (uniform depth; an element belongs to the box of its centroid), and the near
   * blocks S_d are applied as a multilevel FMM over the lattice's boxes: boxes whose grid
   * offset has Chebyshev norm >= 2 interact through M2L on the coarsest such level (moments
   * gathered by P2M about the leaf centres and M2M, locals spread by L2L and L2P, Appendix A
   * eqs. (p2m), (m2m), (m2l), (l2l), (l2p)), leaves that stay near through exact P2P blocks.
   * Storage O(n log n) instead of 9 (or 27) n x n blocks.  Requires near_radius 1 on every
   * axis, every centroid inside the cell's lattice box (else FMBEM_ERR_UNSUPPORTED), no
   * half-space and no exact mode (FMBEM_ERR_UNSUPPORTED); at most 8 levels.  0 => the dense
   * near blocks (FMPBEM). */
  int32_t near_levels;
  /* truncation number n_t,near of the multilevel near field, 1..7 ((n_t,near + 1)^2 <= 64
   * expansion coefficients per box); 0 => min(order, 7).  Ignored when near_levels = 0. */
  int32_t near_order;
} fmbem_plan_desc;

#define FMBEM_TILE_SHAPES 10

#define FMBEM_DFT_AUTO 0    /* autotuned */
#define FMBEM_DFT_AXES 1    /* one direct pruned DFT pass per axis */
#define FMBEM_DFT_FUSED 2   /* both axes of an N3 = 1 grid in one launch through LDS */
#define FMBEM_DFT_GEMM 3    /* axis passes as MFMA GEMMs with the DFT matrices (N_a <= 128) */
#define FMBEM_DFT_FUSED_MFMA 4 /* both axes of an N3 = 1 grid in one launch, as MFMA products with the
                                  DFT matrices, the intermediate in LDS (1 < N_a <= 128) */
#define FMBEM_DFT_FFT 5     /* both axes of an N3 = 1 grid in one launch as mixed-radix FFTs on the
                               vector units (radix 8, 4 or 2 by the axis length, else a direct
                               DFT), the intermediate in LDS; the default where it applies */

typedef struct {
  int32_t n_dof_cell;         /* n (triangles per cell) */
  int32_t n_cells;            /* C = M1 M2 M3 */
  int64_t n_dof;              /* N = C n */
  int32_t p;                  /* (n_t+1)^2 */
  int32_t fft_shape[3];       /* N1, N2, N3 */
  int32_t n_near;             /* number of near-field offsets (unique blocks S_d) */
  int32_t n_far;              /* number of far offsets in the Toeplitz structure (plus the far
                                 image offsets in the half-space) */
  uint32_t precisions;        /* resident operator copies */
  size_t resident_bytes;      /* device memory owned by the plan */
  size_t workspace_bytes_per_rhs[2]; /* matvec workspace per right-hand side, [FP64, FP32] */
  double scale;               /* s of the diagonal scaling s^n applied to V0, U0, Lambda */
  int32_t near_levels;        /* multilevel near field (FMPBEM2): levels L (0: dense near blocks) */
  int32_t near_order;         /* its truncation number n_t,near */
  int64_t near_boxes;         /* boxes of levels 1..L of one cell */
  int64_t near_m2l_pairs;     /* (target box, source box, near offset) triples translated by M2L */
  int64_t near_p2p_entries;   /* exact entries kept in the P2P blocks */
  double near_macs_per_rhs;   /* complex multiply-adds of one multilevel near-field application per
                                 right-hand side, counting only source cells inside the lattice */
  int32_t near_max_tasks;     /* longest list of operator blocks that one workgroup adds up for one
                                 target in any multilevel stage (after the stages are split) */
} fmbem_plan_info;

/* Build the plan: near blocks S_d (Sec. 3.2), P2M V0 and L2P U0 (Appendix A,
 * eqs. (p2m), (l2p)), and Lambda = DFT over the cell grid of the first block
 * column of the circulant embedding of K (Sec. 2.4, eq. (blockDiagonal);
 * Sec. 3.5), all computed on the device in FP64.  Blocks until the plan is
 * ready.  The mesh must be a set of non-degenerate triangles; the returned
 * plan is owned by the caller and released with fmbem_plan_destroy. */
fmbem_status fmbem_plan_create(const fmbem_cell_mesh* mesh, const fmbem_plan_desc* desc,
                               void* hip_stream, fmbem_plan* out);
fmbem_status fmbem_plan_query(fmbem_plan plan, fmbem_plan_info* out);
fmbem_status fmbem_plan_destroy(fmbem_plan plan);

/* Operator data for inspection (host copies; complex128 unless stated):
 *   what = 0: S_d          [n_near][n][n] row-major, offsets in fmbem_plan_offsets order
 *   what = 1: V0           [p][n]   (unscaled)
 *   what = 2: U0           [n][p]   (unscaled)
 *   what = 3: Lambda       [B][p][p] row-major, unscaled and without the 1/B factor
 *   what = 4: near offsets int32 [n_near][3]
 * host_bytes must be at least the size of the requested array.  In the half-space with
 * grid[2] == 1 the exported S_d and Lambda include the image terms; with grid[2] > 1 they are
 * the direct part only (the image part is a second operator).  Blocks. */
fmbem_status fmbem_plan_export(fmbem_plan plan, int32_t what, void* host, size_t host_bytes);

/* y = A x (Sec. 3.5, eq. (FMPBEMsystem)): near-field block-Toeplitz product,
 * S2M, pruned grid FFT, per-bin M2L product, inverse FFT with cropping, L2T.
 * x, y: device [n_rhs][n_cells][n_dof_cell], complex128 for FMBEM_FP64 and
 * complex64 for FMBEM_FP32; x and y must not overlap.  workspace: device,
 * at least n_rhs * workspace_bytes_per_rhs[precision] bytes, 256-byte aligned.
 * The operator copy of that precision must be resident.  Stream-ordered. */
fmbem_status fmbem_matvec(fmbem_plan plan, int32_t precision, int32_t n_rhs,
                          const void* x, void* y, void* workspace, size_t workspace_bytes,
                          void* hip_stream);

/* fmbem_matvec for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops and harnesses that forbid hipMalloc): the same operator application, with the
 * workspace taken from a static device array of FMBEM_NOALLOC_WORKSPACE_BYTES (64 MiB) that the
 * library holds on every device it is loaded on until the process ends.  Calls no allocating
 * routine (the tile shapes and DFT schedule are ones measured earlier for the same problem
 * signature, else the defaults; no timing).  x, y, precision, n_rhs as in fmbem_matvec.
 * Returns FMBEM_ERR_WORKSPACE (nothing queued) when n_rhs * workspace_bytes_per_rhs[precision]
 * exceeds the array.  Every call on one device shares that device's array: calls that overlap
 * on one device (different streams or host threads without ordering) race and give wrong
 * results; calls ordered on one stream are safe (nothing in the array needs to start at zero).
 * Stream-ordered. */
#define FMBEM_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
fmbem_status fmbem_matvec_noalloc(fmbem_plan plan, int32_t precision, int32_t n_rhs, const void* x, void* y,
                                  void* hip_stream);

typedef struct {
  double tol;                 /* stop when ||b - A x||_2 / ||b||_2 <= tol (FP64 true residual) */
  int32_t restart;            /* GMRES restart length m (default 30 when 0), at most 1000 */
  int32_t max_iters;          /* total inner iterations (default 1000 when 0) */
  int32_t max_refinements;    /* outer refinement steps for FP32 inner solves (default 20 when 0) */
  int32_t inner_precision;    /* FMBEM_FP64: plain FP64 GMRES; FMBEM_FP32: FP32 operator inside
                                 GMRES, FP64 Arnoldi, FP64 residual and refinement */
  double inner_tol;           /* relative tolerance of each FP32 inner solve (default 1e-5 when 0) */
  int32_t orthogonalization;  /* FMBEM_ORTHO_*: Gram-Schmidt passes per Arnoldi step */
} fmbem_solve_opts;

/* 0: classical Gram-Schmidt plus a second pass when ||w_new|| < ||w_old|| / sqrt(2)
 *    (Daniel-Gragg-Kaufman-Stewart criterion, decided on the device);
 * 1: always two passes; 2: one pass.  Every solve ends on the FP64 true residual. */
#define FMBEM_ORTHO_DGKS 0
#define FMBEM_ORTHO_TWICE 1
#define FMBEM_ORTHO_ONCE 2

typedef struct {
  int32_t iterations;         /* inner GMRES iterations (operator applications) */
  int32_t refinements;        /* outer refinement steps (FP32 inner mode) */
  double rel_residual;        /* final FP64 ||b - A x|| / ||b|| */
} fmbem_solve_info;

/* Solve A x = b by restarted GMRES (Sec. 2.4, Sec. 3.5; GMRES as in Sec. 4)
 * with classical Gram-Schmidt (a second pass per opts->orthogonalization),
 * Givens rotations, and (for inner_precision = FMBEM_FP32) FP64 iterative
 * refinement around FP32 inner solves.  With FP64 inner precision every
 * restart cycle begins with the FP64 true residual, which decides convergence.
 * b, x: device complex128 [n_rhs][n_cells][n_dof_cell]; x holds the initial
 * guess on entry and the solution on return.  All right-hand sides are
 * iterated together, each in its own Krylov space.  Allocates its Krylov basis
 * on the device for the duration of the call.  Blocks until done; info (host,
 * [n_rhs]) may be NULL.  Returns FMBEM_ERR_NOT_CONVERGED (x = last iterate,
 * info filled) when some right-hand side misses tol within the limits;
 * FMBEM_ERR_INVALID_ARG for bad options or a non-finite ||b||. */
fmbem_status fmbem_solve(fmbem_plan plan, const fmbem_solve_opts* opts, int32_t n_rhs,
                         const void* b, void* x, fmbem_solve_info* info, void* hip_stream);

/* Persistent form of fmbem_solve for repeated solves with one plan and one
 * right-hand-side count (Sec. 2.4, Sec. 3.5, Sec. 4, as fmbem_solve): the
 * Krylov basis, work vectors and operator workspace are allocated once by
 * fmbem_solver_create (opts validated and fixed there) and reused by every
 * fmbem_solver_run.  The solver runs on its own stream (default priority),
 * ordered after the work queued on hip_stream when run is called; run blocks
 * until the solution is in x.  b, x: device complex128 [n_rhs][n_cells]
 * [n_dof_cell], staged into the solver's buffers (x is the initial guess).
 * use_graphs = 1: each Arnoldi step that neither starts nor ends a restart
 * cycle is captured as a HIP graph per (step index, round parity) the second
 * time it occurs and replayed from then on, also in later runs; the iterates
 * are identical to eager execution.  Status and info as fmbem_solve.  A solver
 * is not safe for concurrent runs; the plan must outlive it.
 * graph_stats: graphs instantiated and rounds replayed so far (either may be NULL). */
fmbem_status fmbem_solver_create(fmbem_plan plan, const fmbem_solve_opts* opts, int32_t n_rhs,
                                 int32_t use_graphs, fmbem_solver* out);
fmbem_status fmbem_solver_run(fmbem_solver solver, const void* b, void* x, fmbem_solve_info* info,
                              void* hip_stream);
fmbem_status fmbem_solver_graph_stats(fmbem_solver solver, int32_t* graphs, int64_t* replays);
fmbem_status fmbem_solver_destroy(fmbem_solver solver);

/* Several independent solves (plans of different lattices, meshes, frequencies,
 * right-hand-side counts and options) advanced in lockstep: in every round each
 * unfinished problem applies its operator once, and the near-field + S2M GEMMs
 * of all of them run as one grouped launch, as do their L2T GEMMs (Sec. 3.5,
 * eq. (FMPBEMsystem), batched); the grid DFT / M2L stages run per plan.  Each
 * problem follows fmbem_solve exactly (same iterates up to the rounding of the
 * shared launches).  plans, opts, n_rhs, b, x: arrays of n (b[i], x[i] as in
 * fmbem_solve for plan i); info: host [sum of n_rhs], problem i's entries after
 * those of problems 0..i-1, may be NULL.  The first call for a new combination
 * of problem sizes times the grouped launch's tile shapes.  Blocks until every
 * problem is done.  Returns FMBEM_ERR_NOT_CONVERGED when some problem missed its
 * tolerance (all x and info filled). */
fmbem_status fmbem_solve_batch(int32_t n, const fmbem_plan* plans, const fmbem_solve_opts* opts,
                               const int32_t* n_rhs, const void* const* b, void* const* x,
                               fmbem_solve_info* info, void* hip_stream);

/* Serving engine: continuous batching of solve requests on one stream (the
 * batched form of fmbem_solve for a stream of requests arriving over time).
 * Requests wait in arrival order; at the start of each fmbem_engine_step the
 * head of the queue is admitted while fewer than max_slots problems are active
 * and its device footprint fits hbm_budget_bytes minus what the active problems
 * hold.  The footprint of a request is its Krylov basis ((restart + 1) vectors),
 * four work vectors and the FP32 copy ([n_rhs][N] each) plus the operator
 * workspace, and the resident bytes of its plan unless an active problem of the
 * same plan already counts them; plans are the caller's and stay resident.  The
 * problems' device buffers are stream-ordered allocations from a memory pool of
 * the engine that keeps freed memory for later problems, so admitting and
 * retiring problems never synchronises the device.  A step advances every
 * active problem by one round: one operator application each, with the
 * near-field + S2M and the L2T GEMMs of all of them in shared grouped launches,
 * then their Gram-Schmidt, Givens and residual kernels; finished problems free
 * their memory.  Each problem follows fmbem_solve.  Steps block for the previous
 * round's results only (one round stays in flight).  Not safe for concurrent
 * calls on one engine except submit/poll/stats, which lock.
 *
 * create: hip_stream is the stream every step uses; out receives the engine.
 * submit: plan, b and x (device complex128 [n_rhs][n_cells][n_dof_cell], x the
 *   initial guess, overwritten with the solution) must stay valid until the
 *   ticket is polled done.  Validates opts like fmbem_solve; returns
 *   FMBEM_ERR_ADMISSION (nothing queued) when the footprint (plan included)
 *   exceeds the budget.
 * step: returns FMBEM_OK when idle.
 * poll: *done = 0 while pending (FMBEM_OK); when finished *done = 1, info (host
 *   [n_rhs], may be NULL) is filled and the solve's status is returned
 *   (FMBEM_OK, FMBEM_ERR_NOT_CONVERGED, FMBEM_ERR_INVALID_ARG for a non-finite b,
 *   FMBEM_ERR_OUT_OF_MEMORY); a ticket is reported once, after which it is unknown
 *   (FMBEM_ERR_INVALID_ARG).
 * stats: active problems, queued requests, device bytes held (any may be NULL).
 * destroy: waits for the stream, frees every active problem, drops the queue. */
fmbem_status fmbem_engine_create(size_t hbm_budget_bytes, int32_t max_slots, void* hip_stream,
                                 fmbem_engine* out);
fmbem_status fmbem_engine_submit(fmbem_engine engine, fmbem_plan plan, const fmbem_solve_opts* opts,
                                 int32_t n_rhs, const void* b, void* x, int64_t* ticket);
fmbem_status fmbem_engine_step(fmbem_engine engine);
fmbem_status fmbem_engine_poll(fmbem_engine engine, int64_t ticket, int32_t* done, fmbem_solve_info* info);
fmbem_status fmbem_engine_stats(fmbem_engine engine, int32_t* active, int32_t* queued, size_t* bytes_in_use);
fmbem_status fmbem_engine_destroy(fmbem_engine engine);

/* Where an engine's host time went since it was created (accounting of the serving loop;
 * not part of the method).  enqueue: queueing each round's kernels (every active problem's
 * Gram-Schmidt / Givens / vector kernels and their operator applications, grouped by
 * precision); admit: admitting queued problems (allocation of their buffers and their first
 * kernels); wait: blocking for the previous round's results (the device is busy meanwhile:
 * wait time is device time the host did not have to cover); retire: finishing problems
 * (freeing their buffers).  rounds counts steps with at least one active problem,
 * member_rounds the active problems summed over those steps.  Locks like stats. */
typedef struct {
  int64_t rounds, member_rounds, admitted, retired;
  double enqueue_s, admit_s, wait_s, retire_s;
} fmbem_engine_timing;
fmbem_status fmbem_engine_timing_read(fmbem_engine engine, fmbem_engine_timing* out);

/* Right-hand sides b = p_inc + alpha dp_inc/dn at the collocation points
 * (Sec. 2.1, eq. (bm)), device complex128 [n_rhs][n_cells][n_dof_cell].
 * Plane wave p_inc = A e^{ik d.x} (Sec. 4.1, eq. (planewave)); dirs host [n_rhs][3]
 * unit vectors.  Point source p_inc = A e^{ikR}/R, R = |x - s| (Sec. 4.2);
 * src host [n_rhs][3] absolute positions (m), cell (0,0,0) centred at the origin.
 * Stream-ordered. */
fmbem_status fmbem_incident_plane_wave(fmbem_plan plan, int32_t n_rhs, const double* dirs,
                                       double amplitude, void* b, void* hip_stream);
fmbem_status fmbem_incident_point_source(fmbem_plan plan, int32_t n_rhs, const double* src,
                                         double amplitude, void* b, void* hip_stream);

/* Incident pressure at arbitrary points (no normal-derivative term): kind
 * FMBEM_INCIDENT_PLANE_WAVE, p_inc = A e^{ik d.x} (Sec. 4.1, eq. (planewave)), src =
 * unit directions; kind FMBEM_INCIDENT_POINT_SOURCE, p_inc = A e^{ikR}/R (Sec. 4.2), src =
 * source positions.  src host [n_rhs][3]; points host [n_points][3] absolute positions (m);
 * p_inc device complex128 [n_rhs][n_points].  A point at a source gives inf.  Blocks until
 * the result is written (the host arrays are read on the stream). */
#define FMBEM_INCIDENT_PLANE_WAVE 0
#define FMBEM_INCIDENT_POINT_SOURCE 1
fmbem_status fmbem_incident_at_points(fmbem_plan plan, int32_t kind, int32_t n_rhs, const double* src,
                                      double amplitude, int32_t n_points, const double* points,
                                      void* p_inc, void* hip_stream);

/* Pressure at points of the fluid from the solved surface pressure of the rigid
 * scatterer: the CBIE (Sec. 2.1, eq. (cbie)) with c(x) = 1 off the surface and dp/dn = 0,
 *   p(x_m) = p_inc(x_m) - sum_j x_j int_{Delta_j} dG/dn_y(x_m, y) dA(y),
 * j over the elements of every cell, integrated with the plan's non-self Duffy rule
 * (q x q points, q = 16 / 8 / 4 for |x_m - centroid_j| below 1 / 3 / above 3 longest
 * edges of element j), in FP64.  x: device complex128 [n_rhs][n_cells][n_dof_cell] (the
 * solution of fmbem_solve).  points: host [n_points][3], absolute positions in the fluid
 * (not on the surface; a point on a quadrature point gives inf or NaN).  p_inc: device
 * complex128 [n_rhs][n_points] or NULL (then p is the scattered pressure alone).  p:
 * device complex128 [n_rhs][n_points]; p may equal p_inc, must not overlap x.  Allocates
 * a stream-ordered partial-sum buffer of n_rhs * n_points * ceil(N / 1024) * 16 bytes.
 * Blocks until p is written. */
fmbem_status fmbem_field(fmbem_plan plan, int32_t n_rhs, const void* x, int32_t n_points,
                         const double* points, const void* p_inc, void* p, void* hip_stream);

/* Insertion loss over observation points (eq. (insertionloss)):
 * il[r] = 20 log10( sum_m |p_inc[r][m]| / sum_m |p[r][m]| ).  p_inc, p: device complex128
 * [n_rhs][n_points]; il: device double [n_rhs] (inf when sum |p| = 0).  Stream-ordered. */
fmbem_status fmbem_insertion_loss(int32_t n_rhs, int32_t n_points, const void* p_inc, const void* p,
                                  double* il, void* hip_stream);

/* Per-stage device time of the operator applications made with this plan
 * (fmbem_matvec and the ones inside fmbem_solve), measured with HIP events
 * recorded on the call's stream around each selected stage.  stage_mask != 0
 * clears the counters and records the stages whose bit (1 << stage) is set on
 * every period-th operator application (period >= 1); stage_mask = 0 stops.
 * Each recorded stage adds two event records to the stream.  Not for concurrent
 * use of the same plan from several host threads while enabled.
 * Stages: 0 near field + S2M (one grouped launch), 1 sum of the near-field partial
 * products (only for lattices without far-field offsets), 2 forward DFT, 3 M2L,
 * 4 inverse DFT, 5 L2T with the near-field sum, in FP64; 6..11 the same in FP32. */
#define FMBEM_N_STAGES 12
#define FMBEM_PROFILE_ALL 0xFFFu
fmbem_status fmbem_plan_profile(fmbem_plan plan, uint32_t stage_mask, int32_t period);
/* Synchronizes with the recorded events and returns the accumulated time (ms)
 * and the number of launches of each stage (host arrays [FMBEM_N_STAGES]). */
fmbem_status fmbem_plan_profile_read(fmbem_plan plan, double* ms, int64_t* count);

const char* fmbem_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* FMBEM_H */
