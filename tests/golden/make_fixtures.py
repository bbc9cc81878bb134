"""Writes the stored expected values of the full-size parity tests.

Every value here comes from the FP64 CPU oracle (``oracle/``) applied to the seeded
synthetic inputs of ``workloads/``; nothing is read from the HIP library.

    python tests/golden/make_fixtures.py [grid16_rows] [barrier_rows] [large_cell_rows] [grid16_solution]

Fixtures (NumPy ``.npz``, no pickles):
  grid16_rows.npz        O2 operator (Sec. 3.2 eq. (2dPeriodicFMM), App. A) applied to a
                         seeded random vector on the 16 x 16 lattice of 1280-triangle
                         spheres at 1 kHz, n_t = 10: 288 output rows in corner, edge and
                         interior cells, each computed alone (``operator.sampled_apply``).
  barrier_rows_<f>.npz   the same on the 40 x 2 x 8 lattice of open tube cells at 100 Hz
                         (n_t = 10) and 2 kHz (n_t = 14), 128 rows.
  large_cell_rows.npz    the FMPBEM2 operator (Sec. 3.3: near blocks by the multilevel FMM
                         of ``multilevel.sampled_apply2``, 4 levels, n_t,near = 4) applied
                         to a seeded random vector on the 4 x 4 lattice of 20480-triangle
                         spheres at 1 kHz, n_t = 10: 24 rows in corner, edge and interior
                         cells.
  grid16_solution.npz    solution of the O2 system for the plane-wave right-hand side
                         (Sec. 2.1 eq. (bm), Sec. 4.1 eq. (planewave)) of the same
                         lattice, by the oracle's GMRES(100) to a relative residual of
                         1e-12: every unknown of 12 cells (corners, edges, interior) and
                         the l2 norm of the whole solution.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import bem, operator as op, solve, multilevel as ml  # noqa: E402
from workloads import config_grid16, config_barrier_r4b, config_large_cell  # noqa: E402
from workloads.rng import generator, random_complex  # noqa: E402

# seeds of the random input vectors and of the sampled rows
GRID16_X_SEED = 2201
GRID16_ROW_SEED = 22011
BARRIER_X_SEED = 2202
BARRIER_ROW_SEED = 22021

# 16 x 16 lattice: the four corners, four edge cells and four interior cells
GRID16_CELLS = [(0, 0), (15, 0), (0, 15), (15, 15), (7, 0), (0, 7), (15, 8), (8, 15),
                (7, 7), (8, 8), (3, 12), (12, 3)]
# 40 x 2 x 8 barrier: corners of the lattice, cells on its faces and inside
BARRIER_CELLS = [(0, 0, 0), (39, 1, 7), (0, 1, 7), (39, 0, 0), (20, 0, 0), (20, 1, 7),
                 (19, 0, 4), (21, 1, 3)]


def _cell_index(grid, ijk):
    ijk = tuple(ijk) + (0,) * (3 - len(ijk))
    return ijk[0] + grid[0] * (ijk[1] + grid[1] * ijk[2])


def sampled_dofs(grid, n, cells, per_cell, seed):
    """``per_cell`` elements of every listed cell: the first and last element and
    seeded distinct ones between them."""
    g = generator(seed)
    out = []
    for ijk in cells:
        c = _cell_index(grid, ijk)
        inner = g.choice(np.arange(1, n - 1), per_cell - 2, replace=False)
        rows = np.sort(np.concatenate([[0, n - 1], inner]))
        out.extend(int(c * n + a) for a in rows)
    return np.array(out, dtype=np.int64)


def grid16_rows():
    w = config_grid16()
    n = w.n_dof_cell
    x = random_complex((1, w.lattice.n_cells, n), GRID16_X_SEED)
    dofs = sampled_dofs(w.lattice.grid, n, GRID16_CELLS, 24, GRID16_ROW_SEED)
    y = op.sampled_apply(w.vertices, w.triangles, w.lattice, w.k, w.order, -1j / w.k, x, dofs)
    np.savez(os.path.join(HERE, "grid16_rows.npz"), x_seed=GRID16_X_SEED, dofs=dofs, y=y[0])


def barrier_rows(freq_index):
    w = config_barrier_r4b(freq_index)
    n = w.n_dof_cell
    x = random_complex((1, w.lattice.n_cells, n), BARRIER_X_SEED)
    dofs = sampled_dofs(w.lattice.grid, n, BARRIER_CELLS, 16, BARRIER_ROW_SEED)
    y = op.sampled_apply(w.vertices, w.triangles, w.lattice, w.k, w.order, -1j / w.k, x, dofs)
    name = f"barrier_rows_{int(round(w.frequency))}Hz.npz"
    np.savez(os.path.join(HERE, name), x_seed=BARRIER_X_SEED, freq_index=freq_index, frequency=w.frequency,
             order=w.order, dofs=dofs, y=y[0])


LARGE_X_SEED = 2203
LARGE_ROW_SEED = 22031
LARGE_CELLS = [(0, 0), (3, 3), (0, 3), (1, 0), (3, 2), (1, 1), (2, 2), (2, 1)]


def large_cell_rows():
    w = config_large_cell()
    n = w.n_dof_cell
    x = random_complex((1, w.lattice.n_cells, n), LARGE_X_SEED)
    dofs = sampled_dofs(w.lattice.grid, n, LARGE_CELLS, 3, LARGE_ROW_SEED)
    lv, no = w.extra["near_levels"], w.extra["near_order"]
    y = ml.sampled_apply2(w.vertices, w.triangles, w.lattice, w.k, w.order, -1j / w.k, lv, no, x, dofs)
    np.savez(os.path.join(HERE, "large_cell_rows.npz"), x_seed=LARGE_X_SEED, dofs=dofs, near_levels=lv,
             near_order=no, y=y[0])


def grid16_solution(tol=1e-12):
    w = config_grid16()
    n = w.n_dof_cell
    t0 = time.time()
    F = op.FMPBEM.from_workload(w)
    b = bem.rhs_plane_wave(w.vertices, w.triangles, w.lattice, w.k, -1j / w.k, w.plane_waves)[0]
    print(f"operator blocks {time.time() - t0:.0f} s", flush=True)
    t0 = time.time()
    x, its, res = solve.gmres(F.matvec, b, tol=tol, restart=100, maxiter=1000)
    print(f"GMRES {its} iterations, residual {res:.2e}, {time.time() - t0:.0f} s", flush=True)
    cells = [_cell_index(w.lattice.grid, c) for c in GRID16_CELLS]
    dofs = np.concatenate([np.arange(c * n, (c + 1) * n) for c in cells]).astype(np.int64)
    np.savez(os.path.join(HERE, "grid16_solution.npz"), dofs=dofs, x=x[dofs], norm=np.linalg.norm(x),
             iterations=its, rel_residual=res, tol=tol)


if __name__ == "__main__":
    want = sys.argv[1:] or ["grid16_rows", "barrier_rows", "large_cell_rows", "grid16_solution"]
    for name in want:
        t0 = time.time()
        if name == "grid16_rows":
            grid16_rows()
        elif name == "barrier_rows":
            barrier_rows(0)    # 100 Hz, n_t = 10
            barrier_rows(95)   # 2 kHz, n_t = 14
        elif name == "large_cell_rows":
            large_cell_rows()
        elif name == "grid16_solution":
            grid16_solution()
        else:
            raise SystemExit(f"unknown fixture {name}")
        print(f"{name}: {time.time() - t0:.0f} s", flush=True)
