"""GPU parity of the half-space variant (eq. (green3dHalf), Sec. 2.3, Sec. 3.4, eq. (greenFMMhalfspace))
against the FP64 oracle, through the C ABI.  Tolerances as for the full space: FP64 operator 1e-12,
FP32 operator 1e-5, solution after refinement 1e-6, incident fields and field evaluation 1e-12."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import halfspace as hs, solve
from workloads import Lattice, icosphere, random_complex, unit_directions
from tolerance import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")




CASES = {
    # name: (grid, plane z, R_p, n_t); the sphere of radius 0.1 sits at z = 0 of every cell
    "image_near": ((4, 3, 1), 0.15, 0.7 - 0.3j, 6),
    "image_far": ((5, 3, 1), -0.45, 1.0, 6),
    "all_near_image_far": ((2, 2, 1), -0.5, -1.0, 5),
}


@pytest.fixture(scope="module")
def cases():
    import paper_2201_12050_amd as fm
    v, t = icosphere(1, 0.1)
    k = 2 * np.pi * 700.0 / 343.0
    out = {}
    for name, (grid, zg, rp, nt) in CASES.items():
        lat = Lattice(grid, (0.3, 0.3, 0.3))
        H = hs.FMPBEMHalfSpace(v, t, lat, k, nt, -1j / k, zg, rp)
        P = fm.Plan(v, t, grid, (0.3, 0.3, 0.3), k, nt, halfspace=(zg, rp))
        out[name] = (H, P, lat, zg, rp)
    return v, t, k, out


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("R", [1, 9])
def test_halfspace_matvec_matches_oracle(cases, name, R):
    v, t, k, cs = cases
    H, P, lat, zg, rp = cs[name]
    if name == "all_near_image_far":
        assert P.info["n_far"] == 9  # no direct far offsets, the 9 image offsets through the chain
    x = random_complex((R, lat.n_cells, t.shape[0]), 500 + R)
    ref = H.matvec(x)
    xd = torch.from_numpy(x).cuda()
    assert rel(P.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12
    assert rel(P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5


def test_halfspace_dft_schedules(cases):
    # without the canonical-bin pairing every schedule runs with the D factor off
    import paper_2201_12050_amd as fm
    v, t, k, cs = cases
    H, _, lat, zg, rp = cs["image_near"]
    x = random_complex((9, lat.n_cells, t.shape[0]), 31)
    ref = H.matvec(x)
    xd = torch.from_numpy(x).cuda()
    for sched in ("axes", "fused", "gemm", "mfma", "fft"):
        Q = fm.Plan(v, t, lat.grid, lat.pitch, k, H.order, halfspace=(zg, rp), dft_schedule=sched)
        assert rel(Q.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12, sched
        assert rel(Q.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5, sched
        Q.close()


def test_halfspace_incident_fields(cases):
    v, t, k, cs = cases
    H, P, lat, zg, rp = cs["image_near"]
    dirs = unit_directions(3, 17)
    ref = hs.rhs_plane_wave(v, t, lat, k, -1j / k, dirs, zg, rp)
    assert rel(P.incident_plane_wave(dirs).cpu().numpy().reshape(3, -1), ref) < 1e-12
    src = np.array([[0.3, -1.0, -0.4], [1.0, 1.5, -0.7]])
    ref = hs.rhs_point_source(v, t, lat, k, -1j / k, src, zg, rp, amplitude=2.0)
    assert rel(P.incident_point_source(src, amplitude=2.0).cpu().numpy().reshape(2, -1), ref) < 1e-12


@pytest.mark.parametrize("name", ["image_near", "image_far"])
def test_halfspace_solve_matches_lu(cases, name):
    v, t, k, cs = cases
    H, P, lat, zg, rp = cs[name]
    b = P.incident_plane_wave([[0.6, 0.0, 0.8]])
    x, info = P.solve(b, tol=1e-10, inner="fp32")
    xl = solve.lu_solve(H.dense(), b.cpu().numpy().ravel())
    assert info[0]["rel_residual"] <= 1e-10
    assert rel(x.cpu().numpy().ravel(), xl) < 1e-6


def test_halfspace_field(cases):
    v, t, k, cs = cases
    H, P, lat, zg, rp = cs["image_near"]
    pts = np.array([[0.45, 0.3, -0.25], [1.2, -0.8, -0.05], [0.15, 0.15, 0.12], [0.3, 0.3, -0.11]])
    x = random_complex((2, lat.n_cells, t.shape[0]), 91)
    src = np.array([[0.2, -1.0, -0.3], [0.5, 2.0, -1.0]])
    pin = P.incident_at_points("point_source", src, pts)
    assert rel(pin.cpu().numpy(), hs.incident_point_source_at(pts, k, src, zg, rp)) < 1e-12
    got = P.field(torch.from_numpy(x).cuda(), pts).cpu().numpy()
    ref = hs.field(v, t, lat, k, pts, x.reshape(2, -1), zg, rp)
    assert rel(got, ref) < 1e-12


def test_tubes_standing_on_the_plane():
    # open tube segments whose lower rim lies on a sound-hard plane (the barrier setting of
    # Sec. 4.2 with one layer of cells): image elements touch their originals along the rim
    import paper_2201_12050_amd as fm
    from workloads import tube_segment
    v, t = tube_segment(0.08, 0.25, 32, 3)
    lat = Lattice((3, 2, 1), (0.2, 0.2, 0.25))
    k = 2 * np.pi * 800.0 / 343.0
    zg = float(v[:, 2].min())
    H = hs.FMPBEMHalfSpace(v, t, lat, k, 6, -1j / k, zg, 1.0)
    P = fm.Plan(v, t, lat.grid, lat.pitch, k, 6, halfspace=(zg, 1.0))
    x = random_complex((2, lat.n_cells, t.shape[0]), 77)
    xd = torch.from_numpy(x).cuda()
    ref = H.matvec(x)
    assert rel(P.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12
    assert rel(P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5
    src = np.array([[0.2, -1.5, 0.4]])
    b = P.incident_point_source(src)
    assert rel(b.cpu().numpy().ravel(), hs.rhs_point_source(v, t, lat, k, -1j / k, src, zg, 1.0)[0]) < 1e-12
    xs, info = P.solve(b, tol=1e-10, inner="fp32")
    assert rel(xs.cpu().numpy().ravel(), solve.lu_solve(H.dense(), b.cpu().numpy().ravel())) < 1e-6
    P.close()


@pytest.mark.parametrize("R", [1, 9])
def test_stacked_lattice_over_plane_matches_oracle(R):
    # second case of Sec. 3.4: the lattice is periodic along z, normal to the plane, so the image
    # part is block Hankel along z and runs as a sub-plan on the input reversed along z
    import paper_2201_12050_amd as fm
    v, t = icosphere(1, 0.1)
    lat = Lattice((3, 2, 3), (0.3, 0.3, 0.3))
    k = 2 * np.pi * 600.0 / 343.0
    zg, rp = -0.15, 0.8 + 0.2j
    H = hs.FMPBEMHalfSpace(v, t, lat, k, 6, -1j / k, zg, rp)
    P = fm.Plan(v, t, lat.grid, lat.pitch, k, 6, halfspace=(zg, rp))
    x = random_complex((R, lat.n_cells, t.shape[0]), 640 + R)
    xd = torch.from_numpy(x).cuda()
    ref = H.matvec(x)
    assert rel(P.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12
    assert rel(P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5
    if R == 1:
        b = P.incident_plane_wave([[0.6, 0.0, -0.8]])
        assert rel(b.cpu().numpy().ravel(),
                   hs.rhs_plane_wave(v, t, lat, k, -1j / k, [[0.6, 0.0, -0.8]], zg, rp)[0]) < 1e-12
        xs, info = P.solve(b, tol=1e-10, inner="fp32")
        assert rel(xs.cpu().numpy().ravel(), solve.lu_solve(H.dense(), b.cpu().numpy().ravel())) < 1e-6
        pts = np.array([[0.45, 0.2, 0.75], [1.5, -1.0, 0.1], [0.15, 0.15, -0.05]])
        got = P.field(xs, pts).cpu().numpy()
        assert rel(got, hs.field(v, t, lat, k, pts, xs.cpu().numpy().reshape(1, -1), zg, rp)) < 1e-12
    P.close()


def test_barrier_segments_on_the_plane():
    # open tube segments stacked three high on a sound-hard plane, the lowest rim on the plane
    import paper_2201_12050_amd as fm
    from workloads import tube_segment
    v, t = tube_segment(0.08, 0.25, 32, 3)
    lat = Lattice((4, 2, 3), (0.2, 0.2, 0.25))
    k = 2 * np.pi * 700.0 / 343.0
    zg = float(v[:, 2].min())
    H = hs.FMPBEMHalfSpace(v, t, lat, k, 6, -1j / k, zg, 1.0)
    P = fm.Plan(v, t, lat.grid, lat.pitch, k, 6, halfspace=(zg, 1.0))
    x = random_complex((3, lat.n_cells, t.shape[0]), 78)
    xd = torch.from_numpy(x).cuda()
    ref = H.matvec(x)
    assert rel(P.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12
    assert rel(P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5
    P.close()


def test_halfspace_plans_in_a_batch_and_the_engine():
    # grouped applies: a stacked half-space plan (image sub-plan), a folded one and a full-space
    # plan solved in lockstep, and the same through the serving engine; each as alone
    import paper_2201_12050_amd as fm
    v, t = icosphere(1, 0.1)
    k = 2 * np.pi * 600.0 / 343.0
    plans = [fm.Plan(v, t, (3, 2, 3), (0.3, 0.3, 0.3), k, 6, halfspace=(-0.15, 1.0)),
             fm.Plan(v, t, (4, 3, 1), (0.3, 0.3, 0.3), k, 6, halfspace=(0.15, 0.7 - 0.3j)),
             fm.Plan(v, t, (3, 3, 1), (0.3, 0.3, 0.3), k, 6)]
    bs = [P.incident_plane_wave(unit_directions(2, 40 + i)) for i, P in enumerate(plans)]
    for inner in ("fp64", "fp32"):
        opts = dict(tol=1e-9, inner=inner)
        res = fm.solve_batch([(P, b, None, opts) for P, b in zip(plans, bs)])
        for P, b, (x, infos) in zip(plans, bs, res):
            assert max(i["rel_residual"] for i in infos) <= 1e-9
            xa, _ = P.solve(b, **opts)
            assert rel(x.cpu().numpy(), xa.cpu().numpy()) < 1e-8
    eng = fm.Engine(8 << 30, max_slots=4)
    tickets = [eng.submit(P, b, tol=1e-9, inner="fp32") for P, b in zip(plans, bs)]
    done = {}
    for _ in range(100000):
        eng.step()
        for tk in tickets:
            if tk not in done:
                r = eng.poll(tk)
                if r is not None:
                    done[tk] = r
        if len(done) == len(tickets):
            break
    assert len(done) == len(tickets)
    for P, b, tk in zip(plans, bs, tickets):
        xa, _ = P.solve(b, tol=1e-9, inner="fp32")
        x = done[tk][0] if isinstance(done[tk], tuple) else done[tk]
        assert rel(x.cpu().numpy(), xa.cpu().numpy()) < 1e-8
    eng.close()
    for P in plans:
        P.close()
