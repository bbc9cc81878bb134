"""fmbem_matvec_noalloc (workspace in the library's static device array) against fmbem_matvec
(caller workspace): two calls in a row on each device array, the second with a smaller input,
each compared with the workspace entry point and with the oracle's block-by-block apply."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2201_12050_amd as fm
from paper_2201_12050_amd import _lib
from oracle import operator as op
from workloads import icosphere, Lattice
from workloads.rng import random_complex


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _maxrel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def plans():
    v, t = icosphere(1, 0.1)
    k = 2 * np.pi * 700.0 / 343.0
    out = []
    for grid in ((5, 4, 1), (3, 2, 1)):       # the second call has the smaller input
        lat = Lattice(grid, (0.3, 0.3, 0.3))
        out.append((fm.Plan(v, t, lat.grid, lat.pitch, k, 5), op.FMPBEM(v, t, lat, k, 5, -1j / k), lat, t.shape[0]))
    yield out
    for P, *_ in out:
        P.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_workspace_entry_point(plans, precision):
    torch.cuda.set_device(0)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    tol = 1e-12 if precision == "fp64" else 1e-5
    for (P, F, lat, n), R, seed in zip(plans, (3, 1), (11, 12)):
        print(f"noalloc {precision}: grid {lat.grid}, R {R}, seed {seed}", flush=True)
        x = random_complex((R, lat.n_cells, n), seed)
        xd = torch.from_numpy(x).to(dt).cuda()
        y_ws = P.matvec(xd, precision=precision).cpu().numpy()
        y_na = torch.full_like(xd, float("nan"))
        P.matvec_noalloc(xd, y_na, precision=precision)
        y_na = y_na.cpu().numpy()
        ref = F.matvec(x)
        assert np.isfinite(y_na).all()
        assert _rel(y_na, y_ws) <= tol and _maxrel(y_na, y_ws) <= 10 * tol
        assert _rel(y_na, ref) <= tol and _maxrel(y_na, ref) <= 10 * tol


def test_noalloc_rejects_oversized_workspace():
    torch.cuda.set_device(0)
    v, t = icosphere(2, 0.1)
    P = fm.Plan(v, t, (8, 8, 1), (0.3, 0.3, 0.3), 2 * np.pi * 500.0 / 343.0, 4, precisions=("fp64",))
    per = P.info["workspace_bytes_per_rhs"][0]
    R = _lib.NOALLOC_WORKSPACE_BYTES // per + 1
    x = torch.zeros((R, P.n_cells, P.n), dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(_lib.FmbemError) as e:
        P.matvec_noalloc(x, y, precision="fp64")
    assert e.value.status == 6
    P.close()
