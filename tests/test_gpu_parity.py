"""GPU parity of the HIP library against the FP64 oracle, through the C ABI.

Tolerances (relative l2 norms): FP64 operator 1e-12, FP32 operator 1e-5,
solution after refinement 1e-6; operator data (S_d, V0, U0, Lambda) 1e-12.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bem, operator as op, solve
from workloads import icosphere, tube_segment, Lattice, config_tiny, config_grid16
from workloads.rng import random_complex, unit_directions
from tolerance import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")




def _plan(fm_mod, v, t, grid, pitch, k, nt, formulation="bm"):
    return fm_mod.Plan(v, t, grid, pitch, k, nt, formulation)


CASES = {
    # name: (icosphere level or 'tube', grid, frequency, n_t)
    "sphere80_3x3": (1, (3, 3, 1), 800.0, 6),
    "sphere80_5x3_ragged": (1, (5, 3, 1), 800.0, 4),
    "sphere80_line7": (1, (7, 1, 1), 1200.0, 8),
    "tube192_3x2x3": ("tube", (3, 2, 3), 600.0, 6),
    # n_t = 12: p = 169 > 128 takes the wide form of the M2L GEMV
    "sphere80_4x2_nt12": (1, (4, 2, 1), 1500.0, 12),
}


def _geometry(kind):
    if kind == "tube":
        v, t = tube_segment(0.08, 0.25, 32, 3)
        return v, t, (0.2, 0.2, 0.25)
    v, t = icosphere(kind, 0.1)
    return v, t, (0.3, 0.3, 0.3)


@pytest.fixture(scope="module")
def cases():
    import paper_2201_12050_amd as fm
    out = {}
    for name, (kind, grid, f, nt) in CASES.items():
        v, t, pitch = _geometry(kind)
        lat = Lattice(grid, pitch)
        k = 2 * np.pi * f / 343.0
        F = op.FMPBEM(v, t, lat, k, nt, -1j / k)
        P = fm.Plan(v, t, grid, pitch, k, nt)
        out[name] = (F, P, lat)
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_operator_data_matches_oracle(cases, name):
    F, P, lat = cases[name]
    S = P.export("S")
    offs = P.export("near_offsets")
    assert len(offs) == len(F.near)
    for i, d in enumerate(offs):
        assert rel(S[i], F.S[tuple(int(c) for c in d)]) < 1e-12
    assert rel(P.export("V0"), F.V0) < 1e-12
    assert rel(P.export("U0"), F.U0) < 1e-12
    # Lambda = DFT over the grid of the first block column of the circulant embedding of K
    N = P.info["fft_shape"]
    col = np.zeros((N[2], N[1], N[0], F.p, F.p), dtype=np.complex128)
    for d in F.far:
        col[(d[2] % N[2], d[1] % N[1], d[0] % N[0])] = F.K[d]
    ref = np.fft.fftn(col, axes=(0, 1, 2)).reshape(-1, F.p, F.p)
    assert rel(P.export("Lambda"), ref) < 1e-12


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("R", [1, 3, 9, 32])
def test_matvec_matches_oracle(cases, name, R):
    # R = 9 and 32 take the batched MFMA GEMM form of the per-bin M2L product
    F, P, lat = cases[name]
    x = random_complex((R, lat.n_cells, F.n), 100 + R)
    ref = F.matvec(x)
    xd = torch.from_numpy(x).cuda()
    y64 = P.matvec(xd, precision="fp64").cpu().numpy()
    assert rel(y64, ref) < 1e-12
    y32 = P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy()
    assert rel(y32, ref) < 1e-5
    # every right-hand side on its own
    for r in range(R):
        assert rel(y64[r], ref[r]) < 1e-12


def test_explicit_fft_shape_matches_oracle(cases):
    # the default transform lengths of a lattice with M3 = 1 are 2M (even, self-paired bins at
    # N/2); the minimal odd embedding 2M - 1 and a larger one are exact as well and take the
    # other radices and bin-pairing patterns through the DFT, Lambda and M2L
    import paper_2201_12050_amd as fm
    F, P, lat = cases["sphere80_5x3_ragged"]
    assert P.info["fft_shape"] == (10, 6, 1)
    assert cases["tube192_3x2x3"][1].info["fft_shape"] == (5, 3, 5)
    v, t, pitch = _geometry(1)
    for shape in ((9, 5, 0), (12, 8, 0)):
        Q = fm.Plan(v, t, lat.grid, pitch, F.k, F.order, "bm", fft_shape=shape)
        assert Q.info["fft_shape"] == shape[:2] + (1,)
        for R in (1, 9):
            x = random_complex((R, lat.n_cells, F.n), 300 + R)
            ref = F.matvec(x)
            xd = torch.from_numpy(x).cuda()
            assert rel(Q.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12, shape
            assert rel(Q.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5, shape
        Q.close()


@pytest.mark.parametrize("name", ["sphere80_5x3_ragged", "tube192_3x2x3", "sphere80_4x2_nt12"])
def test_dft_schedules_match_oracle(cases, name):
    # each way of running the grid DFT, forced through the plan descriptor: direct axis passes,
    # the fused two-axis kernel (2-D grids only; the 3-D tube lattice falls back to the passes)
    # the axis passes as MFMA GEMMs with the DFT matrices, both axes fused on the matrix
    # cores and both axes as mixed-radix FFTs (2-D grids only, else the passes)
    import paper_2201_12050_amd as fm
    F, P, lat = cases[name]
    kind = CASES[name][0]
    v, t, pitch = _geometry(kind)
    for R in (1, 9):
        x = random_complex((R, lat.n_cells, F.n), 400 + R)
        ref = F.matvec(x)
        xd = torch.from_numpy(x).cuda()
        out = {}
        for sched in ("axes", "fused", "gemm", "mfma", "fft"):
            Q = fm.Plan(v, t, lat.grid, pitch, F.k, F.order, "bm", dft_schedule=sched)
            out[sched] = Q.matvec(xd, precision="fp64").cpu().numpy()
            assert rel(out[sched], ref) < 1e-12, (sched, R)
            y32 = Q.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy()
            assert rel(y32, ref) < 1e-5, (sched, R)
        # the fused kernel sums in the order of the axis passes: equal bit for bit
        assert np.array_equal(out["axes"], out["fused"])


@pytest.mark.parametrize("name", ["sphere80_line7", "sphere80_4x2_nt12"])
def test_every_tile_shape_matches_oracle(cases, name):
    # every tile shape of the near-field + S2M, L2T and M2L GEMM launches, forced through the plan
    # descriptor (the autotuner runs only the fastest): 24 RHS take the M2L GEMM; p = 81 and 169
    # leave ragged row tiles and a ragged last k step, with enough full k steps for the shapes
    # that keep two steps of loads in flight
    import paper_2201_12050_amd as fm
    F, P, lat = cases[name]
    v, t, pitch = _geometry(CASES[name][0])
    x = random_complex((24, lat.n_cells, F.n), 4242)
    ref = F.matvec(x)
    xd = torch.from_numpy(x).cuda()
    for shape in range(1, 11):
        Q = fm.Plan(v, t, lat.grid, pitch, F.k, F.order, "bm", tile_shape=(shape, shape, shape))
        assert rel(Q.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12, shape
        assert rel(Q.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5, shape
        Q.close()


def test_more_than_256_moments_matches_oracle():
    # n_t = 16: p = 289 > 256 takes the one-row-per-thread form of the M2L GEMV (R = 1, 3) and the
    # M2L GEMM with three row tiles of 128 (R = 9)
    import paper_2201_12050_amd as fm
    v, t = icosphere(1, 0.1)
    lat = Lattice((3, 1, 1), (0.3, 0.3, 0.3))
    k = 2 * np.pi * 2000.0 / 343.0
    F = op.FMPBEM(v, t, lat, k, 16, -1j / k)
    P = fm.Plan(v, t, lat.grid, lat.pitch, k, 16)
    for R in (1, 3, 9):
        x = random_complex((R, lat.n_cells, F.n), 600 + R)
        ref = F.matvec(x)
        xd = torch.from_numpy(x).cuda()
        assert rel(P.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12, R
        assert rel(P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5, R
    P.close()


def test_maximum_order_matches_dense_operator():
    # n_t = 20 (p = 441), the largest order the plan accepts, at 4 kHz (k d = 44 at the far
    # offsets, above 2 n_t): the multipole operator against the dense direct-kernel product within
    # the truncation error of the expansion (the oracle's own multipole apply is 1.1e-6 from it
    # here); FP32 against FP64
    import paper_2201_12050_amd as fm
    v, t = icosphere(1, 0.1)
    lat = Lattice((3, 1, 1), (0.3, 0.3, 0.3))
    k = 2 * np.pi * 4000.0 / 343.0
    A = bem.dense_exact(v, t, lat, k, -1j / k)
    P = fm.Plan(v, t, lat.grid, lat.pitch, k, 20)
    assert P.p == 441
    for R in (1, 9):
        x = random_complex((R, lat.n_cells, t.shape[0]), 700 + R)
        ref = (A @ x.reshape(R, -1).T).T
        xd = torch.from_numpy(x).cuda()
        y64 = P.matvec(xd, precision="fp64").cpu().numpy().reshape(R, -1)
        assert rel(y64, ref) < 1e-5, R
        y32 = P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy().reshape(R, -1)
        assert rel(y32, y64) < 1e-5, R
    P.close()


def test_empty_inputs_are_rejected(tiny):
    # zero and negative counts of right-hand sides or points return FMBEM_ERR_INVALID_ARG before any
    # work is queued, and the plan stays usable
    import ctypes as ct
    from paper_2201_12050_amd import _lib
    w, _, P = tiny["bm"]
    lib = P._lib
    n = w.lattice.n_cells * w.n_dof_cell
    x = torch.zeros((1, n), dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    xp, yp = ct.c_void_p(x.data_ptr()), ct.c_void_p(y.data_ptr())
    for r in (0, -1):
        assert lib.fmbem_matvec(P._h, 0, r, xp, yp, None, 0, None) == 1
        info = (_lib.SolveInfo * 1)()
        assert lib.fmbem_solve(P._h, ct.byref(_lib.solve_opts()), r, xp, yp, info, None) == 1
    pts = np.zeros((1, 3))
    dp = pts.ctypes.data_as(ct.POINTER(ct.c_double))
    assert lib.fmbem_field(P._h, 1, xp, 0, dp, yp, yp, None) == 1
    assert lib.fmbem_insertion_loss(1, 0, yp, yp, yp, None) == 1
    torch.cuda.synchronize()
    xr = torch.from_numpy(random_complex((1, n), 88)).cuda()
    assert rel(P.matvec(xr).cpu().numpy(), P.matvec(xr).cpu().numpy()) == 0.0


def test_dft_mfma_long_axis_matches_oracle():
    # 2 x 40 lattice: 79 bins along axis 1, so the fused matrix-core DFT takes the output tiles of
    # a forward line in two groups and the inverse first pass has more inputs per line than its
    # register sets hold; 3 x 16 = 48 channels (n_t = 3), R = 3
    import paper_2201_12050_amd as fm
    v, t = icosphere(1, 0.1)
    lat = Lattice((2, 40, 1), (0.3, 0.3, 0.3))
    k = 2 * np.pi * 700.0 / 343.0
    F = op.FMPBEM(v, t, lat, k, 3, -1j / k)
    x = random_complex((3, lat.n_cells, t.shape[0]), 911)
    ref = F.matvec(x)
    xd = torch.from_numpy(x).cuda()
    for sched in ("axes", "mfma", "fft"):
        Q = fm.Plan(v, t, lat.grid, lat.pitch, k, 3, "bm", dft_schedule=sched)
        assert rel(Q.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12, sched
        assert rel(Q.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5, sched
        Q.close()


@pytest.mark.parametrize("grid,shape", [((6, 5, 1), (0, 0, 0)), ((4, 3, 1), (0, 0, 0)), ((1, 7, 1), (0, 0, 0)),
                                        ((5, 4, 1), (9, 7, 0)), ((3, 3, 1), (8, 5, 0))])
def test_fft_radices_match_oracle(grid, shape):
    # the mixed-radix FFT schedule over every radix: default lengths 2M give radix 4 x 2 (12 x 10),
    # 8 x 2 (8 x 6) and a single transformed axis (1 x 14); explicit odd lengths take the direct
    # DFT (radix 1) on one or both axes.  Odd channel counts (one RHS, p = 25) move one channel per
    # task, even ones two; 64 RHS fill whole 16-channel slices.
    import paper_2201_12050_amd as fm
    v, t = icosphere(1, 0.1)
    lat = Lattice(grid, (0.3, 0.3, 0.3))
    k = 2 * np.pi * 950.0 / 343.0
    F = op.FMPBEM(v, t, lat, k, 4, -1j / k)
    Q = fm.Plan(v, t, lat.grid, lat.pitch, k, 4, "bm", dft_schedule="fft", fft_shape=shape)
    A = fm.Plan(v, t, lat.grid, lat.pitch, k, 4, "bm", dft_schedule="axes", fft_shape=shape)
    for R in (1, 2, 64):
        x = random_complex((R, lat.n_cells, F.n), 1200 + R)
        ref = F.matvec(x)
        xd = torch.from_numpy(x).cuda()
        y64 = Q.matvec(xd, precision="fp64").cpu().numpy()
        assert rel(y64, ref) < 1e-12, R
        assert rel(Q.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5, R
        # the same operator with the direct axis passes agrees to rounding
        assert rel(y64, A.matvec(xd, precision="fp64").cpu().numpy()) < 1e-13, R
    Q.close()
    A.close()


def test_matvec_batched_equals_alone(cases):
    # below the M2L GEMM threshold every stage computes each column in the same order
    # whatever the batch, so a batched apply equals the single ones bit for bit
    F, P, lat = cases["sphere80_5x3_ragged"]
    x = torch.from_numpy(random_complex((4, lat.n_cells, F.n), 7)).cuda().to(torch.complex64)
    yb = P.matvec(x, precision="fp32")
    for r in range(4):
        ya = P.matvec(x[r:r + 1].contiguous(), precision="fp32")
        assert torch.equal(yb[r:r + 1], ya)
    # from 5 right-hand sides on the M2L product is a GEMM: equal to FP32 rounding
    x = torch.from_numpy(random_complex((12, lat.n_cells, F.n), 8)).cuda().to(torch.complex64)
    yb = P.matvec(x, precision="fp32")
    for r in (0, 7, 11):
        ya = P.matvec(x[r:r + 1].contiguous(), precision="fp32")
        assert (torch.linalg.vector_norm(yb[r] - ya[0]) / torch.linalg.vector_norm(ya)).item() < 1e-6


def test_incident_fields_match_oracle(cases):
    F, P, lat = cases["sphere80_3x3"]
    v, t, _ = _geometry(1)
    dirs = unit_directions(3, 11)
    ref = bem.rhs_plane_wave(v, t, lat, F.k, F.alpha, dirs)
    got = P.incident_plane_wave(dirs).cpu().numpy().reshape(3, -1)
    assert rel(got, ref) < 1e-13
    src = np.array([[0.3, -2.0, 0.1], [1.0, 1.5, -0.7]])
    ref = bem.rhs_point_source(v, t, lat, F.k, F.alpha, src, amplitude=2.0)
    got = P.incident_point_source(src, amplitude=2.0).cpu().numpy().reshape(2, -1)
    assert rel(got, ref) < 1e-13


@pytest.fixture(scope="module")
def tiny():
    import paper_2201_12050_amd as fm
    out = {}
    for form in ("bm", "cbie"):
        w = config_tiny(form)
        F = op.FMPBEM.from_workload(w)
        P = fm.Plan.from_workload(w)
        out[form] = (w, F, P)
    return out


@pytest.mark.parametrize("form", ["bm", "cbie"])
def test_tiny_config_matvec_and_solve(tiny, form):
    # 4x1 line of 320-triangle spheres, 500 Hz, n_t = 10 (N = 1280)
    w, F, P = tiny[form]
    a = bem.default_alpha(w.k, form)
    x = random_complex((1, w.lattice.n_cells, w.n_dof_cell), 3)
    xd = torch.from_numpy(x).cuda()
    assert rel(P.matvec(xd).cpu().numpy(), F.matvec(x)) < 1e-12
    b = bem.rhs_plane_wave(w.vertices, w.triangles, w.lattice, w.k, a, w.plane_waves)
    bd = P.incident_plane_wave(w.plane_waves)
    assert rel(bd.cpu().numpy().reshape(1, -1), b) < 1e-13
    x_lu = solve.lu_solve(F.dense(), b[0])
    xs, info = P.solve(bd, tol=1e-10, inner="fp64")
    assert info[0]["rel_residual"] <= 1e-10
    assert rel(xs.cpu().numpy().ravel(), x_lu) < 1e-8
    xr, info = P.solve(bd, tol=1e-9, inner="fp32")
    assert info[0]["rel_residual"] <= 1e-9
    assert rel(xr.cpu().numpy().ravel(), x_lu) < 1e-6


def test_matvec_many_rhs_matches_oracle(tiny):
    # 832 right-hand sides on the 4x1 line of 320-triangle spheres: thousands of near-field
    # workgroups in one launch and the M2L as a batched GEMM
    w, F, P = tiny["bm"]
    R = 832
    x = random_complex((R, w.lattice.n_cells, w.n_dof_cell), 17)
    ref = F.matvec(x)
    xd = torch.from_numpy(x).cuda()
    assert rel(P.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12
    assert rel(P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5


@pytest.mark.parametrize("ortho", ["once", "twice"])
def test_solve_gram_schmidt_modes(tiny, ortho):
    # every Gram-Schmidt variant reaches the same LU solution (convergence is decided by the
    # FP64 true residual), and an unknown mode is rejected before any work is enqueued
    w, F, P = tiny["bm"]
    b = bem.rhs_plane_wave(w.vertices, w.triangles, w.lattice, w.k, bem.default_alpha(w.k, "bm"),
                           w.plane_waves)
    x_lu = solve.lu_solve(F.dense(), b[0])
    bd = P.incident_plane_wave(w.plane_waves)
    for inner in ("fp64", "fp32"):
        xs, info = P.solve(bd, tol=1e-9, inner=inner, ortho=ortho)
        assert info[0]["rel_residual"] <= 1e-9
        assert rel(xs.cpu().numpy().ravel(), x_lu) < 1e-6
    import paper_2201_12050_amd as fm
    from paper_2201_12050_amd import _lib
    _lib.ORTHO["bogus"] = 7
    try:
        with pytest.raises(fm.FmbemError) as e:
            P.solve(bd, tol=1e-9, ortho="bogus")
        assert e.value.status == 1
    finally:
        del _lib.ORTHO["bogus"]


def test_solve_initial_guess(tiny):
    # a nonzero initial guess takes the operator application of the first true residual (a zero
    # one skips it: A 0 = 0); warm start from the LU solution stops before any iteration; a zero
    # and a nonzero guess in one multi-RHS solve
    w, F, P = tiny["bm"]
    a = bem.default_alpha(w.k, "bm")
    b = bem.rhs_plane_wave(w.vertices, w.triangles, w.lattice, w.k, a, w.plane_waves)
    x_lu = solve.lu_solve(F.dense(), b[0])
    bd = P.incident_plane_wave(w.plane_waves)
    shape = bd.shape
    for inner in ("fp64", "fp32"):
        x0 = torch.from_numpy(random_complex(shape, 31)).cuda()
        xs, info = P.solve(bd, x=x0, tol=1e-9, inner=inner)
        assert info[0]["rel_residual"] <= 1e-9 and rel(xs.cpu().numpy().ravel(), x_lu) < 1e-6
        warm = torch.from_numpy(x_lu.reshape(shape)).cuda()
        xw, info = P.solve(bd, x=warm, tol=1e-9, inner=inner)
        assert info[0]["iterations"] == 0 and info[0]["rel_residual"] <= 1e-9
    b2 = torch.cat([bd, bd]).contiguous()
    x2 = torch.cat([torch.zeros_like(bd), torch.from_numpy(random_complex(shape, 32)).cuda()]).contiguous()
    xs, info = P.solve(b2, x=x2, tol=1e-9, inner="fp32")
    for q in range(2):
        assert info[q]["rel_residual"] <= 1e-9
        assert rel(xs[q].cpu().numpy().ravel(), x_lu) < 1e-6


def test_solve_rejects_non_finite_rhs(tiny):
    import paper_2201_12050_amd as fm
    w, F, P = tiny["bm"]
    bd = P.incident_plane_wave(w.plane_waves)
    bd[0, 1, 2] = complex(float("nan"), 0.0)
    with pytest.raises(fm.FmbemError) as e:
        P.solve(bd, tol=1e-9, inner="fp32")
    assert e.value.status == 1


def test_solve_not_converged_reports_status(tiny):
    w, F, P = tiny["bm"]
    bd = P.incident_plane_wave(w.plane_waves)
    import paper_2201_12050_amd as fm
    with pytest.raises(fm.FmbemError) as e:
        P.solve(bd, tol=1e-14, max_iters=2, inner="fp64")
    assert e.value.status == 5
    xs, info = P.solve(bd, tol=1e-14, max_iters=2, inner="fp64", raise_on_not_converged=False)
    assert info[0]["iterations"] == 2 and np.isfinite(info[0]["rel_residual"])


@pytest.mark.slow
def test_grid16_full_size_sampled_rows():
    # 16x16 lattice of 1280-triangle spheres, 1 kHz, n_t = 10 (N = 327,680), in the launch
    # configuration the benchmark times; sampled output rows computed one by one by the oracle
    import paper_2201_12050_amd as fm
    w = config_grid16()
    P = fm.Plan.from_workload(w)
    x = random_complex((1, w.lattice.n_cells, w.n_dof_cell), 2201)
    xd = torch.from_numpy(x).cuda()
    y64 = P.matvec(xd).cpu().numpy().reshape(1, -1)
    y32 = P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy().reshape(1, -1)
    rng = np.random.default_rng(5)
    n = w.n_dof_cell
    cells = [0, 15, 17 * 8, 255] + list(rng.integers(0, 256, 4))
    dofs = [c * n + int(rng.integers(0, n)) for c in cells]
    ref = op.sampled_apply(w.vertices, w.triangles, w.lattice, w.k, w.order, -1j / w.k, x, dofs)
    assert rel(y64[:, dofs], ref) < 1e-12
    assert rel(y32[:, dofs], ref) < 1e-5


@pytest.mark.parametrize("grid", [(1, 1, 1), (2, 2, 1), (2, 1, 1), (2, 2, 2)])
def test_all_near_lattices_match_oracle(grid):
    # degenerate lattices where every cell pair is in the near field (no far field, no DFT, no
    # M2L): the operator is the near-field block-Toeplitz product alone; a single cell is one
    # dense block.  Matvec in both precisions, and a solve against LU of the dense matrix.
    import paper_2201_12050_amd as fm
    v, t = icosphere(1, 0.1)
    lat = Lattice(grid, (0.3, 0.3, 0.3))
    k = 2 * np.pi * 900.0 / 343.0
    F = op.FMPBEM(v, t, lat, k, 4, -1j / k)
    P = fm.Plan(v, t, grid, (0.3, 0.3, 0.3), k, 4)
    assert P.info["n_far"] == 0
    x = random_complex((3, lat.n_cells, t.shape[0]), 70 + lat.n_cells)
    ref = F.matvec(x)
    xd = torch.from_numpy(x).cuda()
    assert rel(P.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12
    assert rel(P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5
    b = P.incident_plane_wave([[0.0, 0.6, 0.8]])
    xs, info = P.solve(b, tol=1e-10, inner="fp32")
    xl = solve.lu_solve(bem.dense_exact(v, t, lat, k, -1j / k), b.cpu().numpy().ravel())
    assert info[0]["rel_residual"] <= 1e-10
    assert rel(xs.cpu().numpy().ravel(), xl) < 1e-6
    P.close()


def test_wider_near_field_matches_oracle():
    # near radius 2 on a 6 x 5 lattice: 25 near blocks, the far field starts two cells away
    import paper_2201_12050_amd as fm
    v, t = icosphere(1, 0.1)
    lat = Lattice((6, 5, 1), (0.3, 0.3, 0.3))
    k = 2 * np.pi * 1100.0 / 343.0
    F = op.FMPBEM(v, t, lat, k, 6, -1j / k, near_radius=(2, 2, 2))
    P = fm.Plan(v, t, lat.grid, lat.pitch, k, 6, near_radius=(2, 2, 2))
    assert P.info["n_near"] == 25
    x = random_complex((2, lat.n_cells, t.shape[0]), 808)
    ref = F.matvec(x)
    xd = torch.from_numpy(x).cuda()
    assert rel(P.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12
    assert rel(P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5
    P.close()
