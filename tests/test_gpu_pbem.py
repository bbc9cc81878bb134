"""The exact periodic BEM (PBEM, the paper's comparison method: every block integrated, the
circulant embedding applied with n x n blocks per bin) on the GPU against the oracle's dense
exact collocation matrix O1 (oracle.bem.dense_exact, every block from absolute coordinates),
through the C ABI.  Tolerances: FP64 operator 1e-12, FP32 1e-5, solutions 1e-6 (relative l2
and max-norm)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bem, solve
from workloads import icosphere, tube_segment, Lattice, config_tiny
from workloads.rng import random_complex
from tolerance import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


CASES = {
    # name: (geometry, grid, frequency)
    "sphere80_3x2": ("sphere1", (3, 2, 1), 900.0),
    "sphere80_1x1": ("sphere1", (1, 1, 1), 700.0),
    "sphere80_line5": ("sphere1", (5, 1, 1), 1300.0),
    "tube192_2x2x2": ("tube", (2, 2, 2), 600.0),
}


def _geometry(kind):
    if kind == "tube":
        v, t = tube_segment(0.08, 0.25, 32, 3)
        return v, t, (0.2, 0.2, 0.25)
    v, t = icosphere(1, 0.1)
    return v, t, (0.3, 0.3, 0.3)


@pytest.mark.parametrize("name", list(CASES))
def test_exact_matvec_matches_dense_bem(name):
    import paper_2201_12050_amd as fm
    kind, grid, f = CASES[name]
    v, t, pitch = _geometry(kind)
    lat = Lattice(grid, pitch)
    k = 2 * np.pi * f / 343.0
    A = bem.dense_exact(v, t, lat, k, -1j / k)
    P = fm.Plan(v, t, grid, pitch, k, 0, exact=True)
    n = t.shape[0]
    assert P.p == n and P.info["n_near"] == 0
    for R in (1, 3, 9):   # 9 takes the batched MFMA GEMM of the per-bin product
        x = random_complex((R, lat.n_cells, n), 1500 + R)
        ref = (x.reshape(R, -1) @ A.T).reshape(x.shape)
        xd = torch.from_numpy(x).cuda()
        assert rel(P.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12, R
        assert rel(P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5, R
    P.close()


@pytest.mark.parametrize("formulation", ["bm", "cbie"])
def test_exact_solve_tiny_matches_lu(formulation):
    # the tiny workload (4 x 1 line of 320-triangle spheres, 500 Hz): PBEM solves equal the
    # dense LU solution of the collocation system
    import paper_2201_12050_amd as fm
    w = config_tiny(formulation)
    alpha = bem.default_alpha(w.k, formulation)
    A = bem.dense_exact(w.vertices, w.triangles, w.lattice, w.k, alpha)
    b = bem.rhs_plane_wave(w.vertices, w.triangles, w.lattice, w.k, alpha, w.plane_waves)[0]
    xl = solve.lu_solve(A, b)
    P = fm.Plan(w.vertices, w.triangles, w.lattice.grid, w.lattice.pitch, w.k, 0, formulation, exact=True)
    bd = P.incident_plane_wave(w.plane_waves)
    assert rel(bd.cpu().numpy().ravel(), b) < 1e-13
    for inner in ("fp64", "fp32"):
        xs, info = P.solve(bd, tol=1e-10, inner=inner)
        assert info[0]["rel_residual"] <= 1e-10
        assert rel(xs.cpu().numpy().ravel(), xl) < 1e-6, inner
    P.close()


def test_exact_rejects_halfspace():
    import paper_2201_12050_amd as fm
    v, t = icosphere(1, 0.1)
    with pytest.raises(fm.FmbemError) as e:
        fm.Plan(v, t, (2, 2, 1), (0.3, 0.3, 0.3), 10.0, 0, exact=True, halfspace=(-0.15, 1.0))
    assert e.value.status == 2
