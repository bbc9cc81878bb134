"""GPU parity of the post-processing entry points against the FP64 oracle, through the
C ABI: incident pressure at points, pressure at points of the fluid (eq. (cbie) with
c = 1) and the insertion loss (eq. (insertionloss)).  Tolerance 1e-12 (relative l2):
the same FP64 quadrature on both sides, summed in a different order."""
import ctypes as ct

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bem
from workloads import Lattice, config_barrier_r4b, icosphere, random_complex, tube_segment, unit_directions
from tolerance import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")




def _sphere_points(lat, rng):
    """Points far from the lattice, between cells, close to a sphere (Duffy rules 16 and 8)
    and inside spheres (where the representation gives the extinguished field)."""
    far = np.array([[0.6, -1.5, 0.4], [3.0, 2.0, -1.0], [-2.0, 0.3, 0.0]])
    between = np.array([lat.cell_origin(c) + [0.15, 0.15, 0.0] for c in (0, 4, 7)])
    d = rng.normal(size=(6, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    close = np.array([lat.cell_origin(c) for c in (1, 6, 13, 2, 9, 14)]) + d * np.array(
        [0.101, 0.104, 0.11, 0.13, 0.16, 0.2])[:, None]
    inside = np.array([lat.cell_origin(c) + [0.02, -0.03, 0.01] for c in (3, 10)])
    return np.vstack([far, between, close, inside])


@pytest.fixture(scope="module")
def spheres():
    import paper_2201_12050_amd as fm
    v, t = icosphere(1, 0.1)
    lat = Lattice((5, 3, 1), (0.3, 0.3, 0.3))   # N = 1200: two element chunks, ragged tail
    k = 2 * np.pi * 800.0 / 343.0
    P = fm.Plan(v, t, lat.grid, lat.pitch, k, 4)
    return v, t, lat, k, P


@pytest.mark.parametrize("R", [1, 5])
def test_field_matches_oracle(spheres, R):
    v, t, lat, k, P = spheres
    pts = _sphere_points(lat, np.random.default_rng(7))
    x = random_complex((R, lat.n_cells, t.shape[0]), 31 + R)
    dirs = unit_directions(R, 5)
    xd = torch.from_numpy(x).cuda()
    pin = P.incident_at_points("plane_wave", dirs, pts)
    got = P.field(xd, pts, pin).cpu().numpy()
    ref = bem.field(v, t, lat, k, pts, x.reshape(R, -1), bem.incident_plane_wave_at(pts, k, dirs))
    assert rel(got, ref) < 1e-12
    # the scattered part alone (no incident field given)
    got_s = P.field(xd, pts).cpu().numpy()
    ref_s = bem.field(v, t, lat, k, pts, x.reshape(R, -1))
    assert rel(got_s, ref_s) < 1e-12
    for r in range(R):  # each right-hand side on its own, not just the stack
        assert rel(got_s[r], ref_s[r]) < 1e-12


def test_field_tube_lattice_three_axes():
    import paper_2201_12050_amd as fm
    v, t = tube_segment(0.08, 0.25, 32, 3)
    lat = Lattice((3, 2, 3), (0.2, 0.2, 0.25))   # N = 3456: four chunks, the last ragged
    k = 2 * np.pi * 600.0 / 343.0
    P = fm.Plan(v, t, lat.grid, lat.pitch, k, 6)
    pts = np.array([[0.1, -1.0, 0.3], [0.1, 0.1, 0.25], [0.2, 0.2, 0.2],   # far, between tubes, on a tube axis
                    [0.0, 0.0, 0.0], [0.2, 0.09, 0.5], [-0.5, 0.6, 1.2], [0.4, 0.2, 0.6]])
    x = random_complex((3, lat.n_cells, t.shape[0]), 77)
    src = np.array([[0.2, -2.0, 0.25], [1.0, 1.0, 2.0], [-1.0, 0.0, 0.3]])
    pin = P.incident_at_points("point_source", src, pts, amplitude=2.0)
    got = P.field(torch.from_numpy(x).cuda(), pts, pin).cpu().numpy()
    ref = bem.field(v, t, lat, k, pts, x.reshape(3, -1), bem.incident_point_source_at(pts, k, src, 2.0))
    assert rel(got, ref) < 1e-12


def test_field_output_may_alias_incident(spheres):
    import paper_2201_12050_amd as fm
    v, t, lat, k, P = spheres
    pts = _sphere_points(lat, np.random.default_rng(8))
    x = random_complex((2, lat.n_cells, t.shape[0]), 40)
    xd = torch.from_numpy(x).cuda()
    pin = P.incident_at_points("plane_wave", unit_directions(2, 9), pts)
    want = P.field(xd, pts, pin).cpu().numpy()
    lib = fm.load()
    buf = pin.clone()
    c_pts = np.ascontiguousarray(pts)
    st = lib.fmbem_field(P._h, 2, ct.c_void_p(xd.data_ptr()), pts.shape[0],
                         c_pts.ctypes.data_as(ct.POINTER(ct.c_double)), ct.c_void_p(buf.data_ptr()),
                         ct.c_void_p(buf.data_ptr()), None)
    assert st == 0
    assert np.array_equal(buf.cpu().numpy(), want)


def test_incident_at_points_matches_oracle(spheres):
    _, _, lat, k, P = spheres
    pts = _sphere_points(lat, np.random.default_rng(9))
    dirs = unit_directions(3, 12)
    got = P.incident_at_points("plane_wave", dirs, pts, amplitude=1.5).cpu().numpy()
    assert rel(got, bem.incident_plane_wave_at(pts, k, dirs, 1.5)) < 1e-13
    src = np.array([[0.3, -2.0, 0.1], [1.0, 1.5, -0.7]])
    got = P.incident_at_points("point_source", src, pts, amplitude=2.0).cpu().numpy()
    assert rel(got, bem.incident_point_source_at(pts, k, src, 2.0)) < 1e-13


def test_insertion_loss_matches_oracle():
    import paper_2201_12050_amd as fm
    pin = random_complex((3, 300), 3)
    p = random_complex((3, 300), 4) * np.array([[1.0], [0.1], [3.0]])
    got = fm.insertion_loss(torch.from_numpy(pin).cuda(), torch.from_numpy(p).cuda()).cpu().numpy()
    assert np.allclose(got, bem.insertion_loss(pin, p), rtol=0, atol=1e-12)
    one = fm.insertion_loss(torch.from_numpy(pin[0]).cuda(), torch.from_numpy(0.5 * pin[0]).cuda()).cpu().numpy()
    assert np.allclose(one, 20 * np.log10(2.0), atol=1e-12)


def test_field_rejects_bad_points(spheres):
    import paper_2201_12050_amd as fm
    _, t, lat, _, P = spheres
    xd = torch.zeros((1, lat.n_cells, t.shape[0]), dtype=torch.complex128, device="cuda")
    with pytest.raises(fm.FmbemError):
        P.field(xd, np.array([[0.0, np.nan, 0.0]]))
    with pytest.raises(ValueError):
        P.field(xd.to(torch.complex64), np.zeros((1, 3)))


def test_barrier_receivers_full_size_sampled():
    # barrier lattice 40 x 2 x 8 of open tube cells (N = 122,880) at 100 Hz, all 64 receivers
    # in one launch as the benchmark makes it; four receivers computed one by one by the oracle
    import paper_2201_12050_amd as fm
    w = config_barrier_r4b(0)
    P = fm.Plan.from_workload(w, precisions=("fp64",))
    rec = w.extra["receivers"]
    x = random_complex((1, w.lattice.n_cells, w.n_dof_cell), 2026)
    xd = torch.from_numpy(x).cuda()
    pin = P.incident_at_points("point_source", w.point_sources, rec)
    got_s = P.field(xd, rec).cpu().numpy()   # the scattered part: the incident field would mask it
    got = P.field(xd, rec, pin)
    il = fm.insertion_loss(pin, got).cpu().numpy()
    pick = [0, 27, 36, 63]
    ref_s = bem.field(w.vertices, w.triangles, w.lattice, w.k, rec[pick], x.reshape(1, -1))
    assert rel(got_s[:, pick], ref_s) < 1e-12
    ref_in = bem.incident_point_source_at(rec, w.k, w.point_sources)
    assert rel(got.cpu().numpy(), ref_in + got_s) < 1e-13
    assert np.allclose(il, bem.insertion_loss(ref_in, ref_in + got_s), atol=1e-12)
    P.close()
