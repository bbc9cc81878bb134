"""Pins for oracle.solve and the whole BEM: GMRES vs LU, Mie series convergence."""
import numpy as np
import pytest

from oracle import bem, mie, solve, operator as op
from workloads import icosphere, Lattice, config_tiny


def test_gmres_matches_lu():
    rng = np.random.default_rng(0)
    n = 120
    A = np.eye(n) * 2 + (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) / np.sqrt(4 * n)
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    x_lu = solve.lu_solve(A, b)
    x, its, rel = solve.gmres(lambda v: A @ v, b, tol=1e-13, restart=20)
    assert rel <= 1e-13
    assert np.linalg.norm(x - x_lu) <= 1e-11 * np.linalg.norm(x_lu)
    assert its > 20  # exercised at least one restart


def _mie_error(level, f, formulation):
    v, t = icosphere(level, 0.1)
    lat = Lattice((1, 1, 1), (0.3, 0.3, 0.3))
    k = 2 * np.pi * f / 343.0
    a = bem.default_alpha(k, formulation)
    A = bem.dense_exact(v, t, lat, k, a)
    b = bem.rhs_plane_wave(v, t, lat, k, a, [[1.0, 0.0, 0.0]])[0]
    x = solve.lu_solve(A, b)
    g = bem.element_geometry(v, t)
    ex = mie.rigid_sphere_surface_pressure(g["centroid"], 0.1, k)
    w = g["area"]
    return np.sqrt((w * abs(x - ex) ** 2).sum() / (w * abs(ex) ** 2).sum())


@pytest.mark.parametrize("formulation", ["bm", "cbie"])
def test_mie_convergence(formulation):
    # surface pressure of one rigid sphere converges to the Mie series under refinement;
    # bounds calibrated once (level 1: 80, level 2: 320 triangles)
    e1 = _mie_error(1, 500.0, formulation)
    e2 = _mie_error(2, 500.0, formulation)
    assert e2 < e1 / 2.5
    assert e1 < 0.04 and e2 < 0.012


def test_mie_series_is_solution_of_helmholtz_limit():
    # at ka -> 0 the rigid sphere barely scatters: surface pressure -> incident field, p = 1 + O(ka)
    pts = np.array([[0.1, 0, 0], [0, 0.1, 0], [-0.1, 0, 0]])
    p = mie.rigid_sphere_surface_pressure(pts, 0.1, 1e-3)
    assert np.allclose(p, 1.0, atol=1e-3)


@pytest.mark.slow
def test_tiny_config_gmres_vs_lu():
    # 4x1 line of 320-triangle spheres, 500 Hz, n_t = 10: GMRES on O2 reaches 1e-10, LU on dense O2 agrees
    w = config_tiny()
    F = op.FMPBEM.from_workload(w)
    a = bem.default_alpha(w.k, w.formulation)
    b = bem.rhs_plane_wave(w.vertices, w.triangles, w.lattice, w.k, a, w.plane_waves)[0]
    x_lu = solve.lu_solve(F.dense(), b)
    x, its, rel = solve.gmres(F.matvec, b, tol=1e-12, restart=50)
    assert rel <= 1e-12
    assert np.linalg.norm(x - x_lu) <= 1e-10 * np.linalg.norm(x_lu)
