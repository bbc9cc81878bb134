"""Persistent solver (buffers reused across solves, optional HIP-graph replay of Arnoldi
steps) through the C ABI: every run, eager or replayed, equals fmbem_solve bit for bit (same
kernels in the same order), graphs are replayed across runs with unrelated eager work and
synchronisations in between, and the solution matches the oracle's dense LU (1e-6)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bem, operator as op, solve
from workloads import config_tiny, icosphere, Lattice
from workloads.rng import unit_directions
from tolerance import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")




@pytest.fixture(scope="module")
def case():
    import paper_2201_12050_amd as fm
    v, t = icosphere(1, 0.1)
    grid, pitch, f, nt, R = (4, 3, 1), (0.3, 0.3, 0.3), 1300.0, 8, 2
    lat = Lattice(grid, pitch)
    k = 2 * np.pi * f / 343.0
    a = -1j / k
    F = op.FMPBEM(v, t, lat, k, nt, a)
    P = fm.Plan(v, t, grid, pitch, k, nt)
    Ad = F.dense()
    rhs = []
    for seed in (1, 2, 3):
        dirs = unit_directions(R, 500 + seed)
        b = bem.rhs_plane_wave(v, t, lat, k, a, dirs)
        rhs.append((P.incident_plane_wave(dirs), np.stack([solve.lu_solve(Ad, b[q]) for q in range(R)])))
    return P, R, rhs


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_solver_runs_equal_solve_and_replay_graphs(case, inner):
    import paper_2201_12050_amd as fm
    P, R, rhs = case
    # a short restart so that every run has several cycles, hence replayed steps
    opts = dict(tol=1e-10, restart=6, inner=inner, ortho="dgks")
    eager = fm.Solver(P, R, graphs=False, **opts)
    graph = fm.Solver(P, R, graphs=True, **opts)
    y = torch.zeros_like(rhs[0][0])
    for rep in range(2):
        for b, x_lu in rhs:
            xs, infs = P.solve(b, **opts)
            xe, infe = eager.run(b)
            xg, infg = graph.run(b)
            assert torch.equal(xe, xs) and infe == infs
            assert torch.equal(xg, xs) and infg == infs
            assert rel(xg.cpu().numpy().reshape(x_lu.shape), x_lu) < 1e-6
            # unrelated eager work and a synchronisation between graph replays
            P.matvec(b, y)
            y.mul_(0.5)
            torch.cuda.synchronize()
    st = graph.graph_stats()
    assert st["graphs"] > 0 and st["replays"] > 0
    assert eager.graph_stats() == dict(graphs=0, replays=0)
    eager.close()
    graph.close()


def test_solver_rejects_mismatched_rhs_and_bad_opts(case):
    import paper_2201_12050_amd as fm
    P, R, rhs = case
    with pytest.raises(fm.FmbemError) as e:
        fm.Solver(P, R, tol=0.0)
    assert e.value.status == 1
    sv = fm.Solver(P, 1, tol=1e-8)
    with pytest.raises(ValueError):
        sv.run(rhs[0][0])  # two right-hand sides for a one-RHS solver
    sv.close()
