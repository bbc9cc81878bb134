"""Full-size parity against stored oracle values (tests/golden, written by
tests/golden/make_fixtures.py from the FP64 oracle alone), in the launch configuration
the benchmark times.

* 16 x 16 lattice of 1280-triangle spheres, 1 kHz, n_t = 10 (N = 327,680): 288 rows of
  the operator applied to a seeded vector (corner, edge and interior cells), FP64 <= 1e-12
  and FP32 <= 1e-5; the solution of the plane-wave problem after FP32-refined and FP64
  solves to the benchmark's residual target, <= 1e-6 on every unknown of 12 cells.
* 40 x 2 x 8 barrier of open tube cells at 100 Hz (n_t = 10) and 2 kHz (n_t = 14):
  128 rows of the operator (the three-axis grid transform, the 225-row M2L of n_t = 14,
  and the FP32 dynamic range at the lowest frequency).
* 4 x 4 lattice of 20480-triangle spheres, 1 kHz, n_t = 10, multilevel near field of 4
  levels with n_t,near = 4 (FMPBEM2, N = 327,680): 24 rows of the operator applied to a
  seeded vector, FP64 <= 1e-12 and FP32 <= 1e-5.

Each bound holds for the relative l2 error and for the max-norm error relative to the
largest reference entry."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import config_grid16, config_barrier_r4b, config_large_cell
from workloads.rng import random_complex
from tolerance import rel

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _load(name):
    return np.load(os.path.join(GOLDEN, name), allow_pickle=False)


@pytest.fixture(scope="module")
def grid16():
    import paper_2201_12050_amd as fm
    w = config_grid16()
    P = fm.Plan.from_workload(w)
    yield w, P
    P.close()


def _rows(P, w, fx):
    x = random_complex((1, w.lattice.n_cells, w.n_dof_cell), int(fx["x_seed"]))
    xd = torch.from_numpy(x).cuda()
    ws64, ws32 = P.workspace(1, "fp64"), P.workspace(1, "fp32")
    y64 = P.matvec(xd, None, "fp64", ws64).cpu().numpy().ravel()
    y32 = P.matvec(xd.to(torch.complex64), None, "fp32", ws32).cpu().numpy().ravel()
    dofs = fx["dofs"]
    return y64[dofs], y32[dofs]


def test_grid16_sampled_rows_match_oracle(grid16):
    w, P = grid16
    fx = _load("grid16_rows.npz")
    assert fx["dofs"].size >= 256
    y64, y32 = _rows(P, w, fx)
    e64, e32 = rel(y64, fx["y"]), rel(y32, fx["y"])
    print(f"grid16 rows: fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 < 1e-12
    assert e32 < 1e-5


@pytest.mark.parametrize("name,freq_index", [("barrier_rows_100Hz.npz", 0), ("barrier_rows_2000Hz.npz", 95)])
def test_barrier_sampled_rows_match_oracle(name, freq_index):
    import paper_2201_12050_amd as fm
    fx = _load(name)
    w = config_barrier_r4b(freq_index)
    assert int(fx["order"]) == w.order and abs(float(fx["frequency"]) - w.frequency) < 1e-9
    P = fm.Plan.from_workload(w)
    try:
        y64, y32 = _rows(P, w, fx)
    finally:
        P.close()
    e64, e32 = rel(y64, fx["y"]), rel(y32, fx["y"])
    print(f"barrier {w.frequency:.0f} Hz rows: fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 < 1e-12
    assert e32 < 1e-5


@pytest.mark.parametrize("inner", ["fp32", "fp64"])
def test_grid16_solution_matches_oracle(grid16, inner):
    import paper_2201_12050_amd as fm
    w, P = grid16
    fx = _load("grid16_solution.npz")
    b = P.incident_plane_wave(w.plane_waves)
    # the benchmark's solver and residual target (FP64 true relative residual 1e-7)
    sv = fm.Solver(P, 1, tol=1e-7, inner=inner, ortho="once")
    try:
        x, info = sv.run(b)
        xs = x.cpu().numpy().ravel()
    finally:
        sv.close()
    assert info[0]["rel_residual"] <= 1e-7
    e = rel(xs[fx["dofs"]], fx["x"])
    en = abs(np.linalg.norm(xs) - float(fx["norm"])) / float(fx["norm"])
    print(f"grid16 solution ({inner}): sampled cells {e:.2e}, norm {en:.2e}, {info[0]}")
    assert e < 1e-6
    assert en < 1e-6


def test_large_cell_multilevel_rows_match_oracle():
    import paper_2201_12050_amd as fm
    w = config_large_cell()
    fx = _load("large_cell_rows.npz")
    P = fm.Plan.from_workload(w, near_levels=int(fx["near_levels"]), near_order=int(fx["near_order"]))
    assert P.info["n_near"] == 0 and P.info["near_levels"] == int(fx["near_levels"])
    y64, y32 = _rows(P, w, fx)
    e64, e32 = rel(y64, fx["y"]), rel(y32, fx["y"])
    print(f"large-cell FMPBEM2 rows: fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 < 1e-12
    assert e32 < 1e-5
    P.close()
