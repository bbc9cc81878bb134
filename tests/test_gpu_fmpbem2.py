"""FMPBEM2 (Sec. 3.3: the near blocks as a multilevel FMM over the boxes of the lattice) on
the GPU against the oracle's FMPBEM2 (oracle.multilevel: every near block composed leaf pair
by leaf pair from the exact entries and the P2M / M2M / M2L / L2L / L2P chain), through the C
ABI.  Tolerances: FP64 operator 1e-12, FP32 1e-5 (relative l2 and max-norm), solutions 1e-8
against the oracle's LU of the same operator."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bem, solve, multilevel as ml
from workloads import icosphere, tube_segment, Lattice
from workloads.rng import random_complex, unit_directions
from tolerance import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


CASES = {
    # name: (geometry, grid, frequency, n_t, levels, n_t,near)
    "sphere80_3x3_L2": ("sphere1", (3, 3, 1), 900.0, 6, 2, 4),
    "sphere320_4x3_L2": ("sphere2", (4, 3, 1), 700.0, 6, 2, 5),
    "sphere320_5x1_L3": ("sphere2", (5, 1, 1), 1300.0, 8, 3, 6),
    "sphere80_1x1_L2": ("sphere1", (1, 1, 1), 600.0, 4, 2, 4),      # no far field
    "tube192_2x2x2_L1": ("tube", (2, 2, 2), 600.0, 6, 1, 7),        # 27 near offsets
    "sphere80_3x1_L4_nt1": ("sphere1", (3, 1, 1), 800.0, 5, 4, 1),  # deep tree, lowest order
    "sphere80_4x2_100Hz": ("sphere1", (4, 2, 1), 100.0, 6, 2, 7),   # FP32 range, highest order
}


def _geometry(kind):
    if kind == "tube":
        v, t = tube_segment(0.08, 0.25, 32, 3)
        return v, t, (0.2, 0.2, 0.25)
    v, t = icosphere(int(kind[-1]), 0.1)
    return v, t, (0.3, 0.3, 0.3)


_ORACLE = {}


def _case(name):
    if name not in _ORACLE:
        kind, grid, f, nt, levels, ntn = CASES[name]
        v, t, pitch = _geometry(kind)
        lat = Lattice(grid, pitch)
        k = 2 * np.pi * f / 343.0
        F = ml.FMPBEM2(v, t, lat, k, nt, -1j / k, levels, ntn)
        _ORACLE[name] = (v, t, lat, k, F, F.dense())
    return _ORACLE[name]


@pytest.mark.parametrize("name", list(CASES))
def test_multilevel_matvec_matches_oracle(name):
    import paper_2201_12050_amd as fm
    v, t, lat, k, F, A = _case(name)
    _, grid, _, nt, levels, ntn = CASES[name]
    P = fm.Plan(v, t, grid, lat.pitch, k, nt, near_levels=levels, near_order=ntn)
    assert P.info["n_near"] == 0
    n = t.shape[0]
    for R in (1, 3, 9):   # column tiles of 16, 32 and 64 (R C columns), GEMV and GEMM M2L
        x = random_complex((R, lat.n_cells, n), 2200 + R)
        ref = (x.reshape(R, -1) @ A.T).reshape(x.shape)
        xd = torch.from_numpy(x).cuda()
        assert rel(P.matvec(xd, precision="fp64").cpu().numpy(), ref) < 1e-12, R
        assert rel(P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy(), ref) < 1e-5, R
    P.close()


def test_multilevel_differs_from_dense_near_field_by_the_truncation():
    # the same plan with dense near blocks: the two operators differ by the multilevel
    # approximation of the near blocks alone (oracle: S~_d - S_d)
    import paper_2201_12050_amd as fm
    v, t, lat, k, F, A = _case("sphere320_4x3_L2")
    _, grid, _, nt, levels, ntn = CASES["sphere320_4x3_L2"]
    P2 = fm.Plan(v, t, grid, lat.pitch, k, nt, near_levels=levels, near_order=ntn)
    P1 = fm.Plan(v, t, grid, lat.pitch, k, nt)
    x = random_complex((2, lat.n_cells, t.shape[0]), 77)
    xd = torch.from_numpy(x).cuda()
    diff = (P2.matvec(xd, precision="fp64") - P1.matvec(xd, precision="fp64")).cpu().numpy()
    ref = np.zeros_like(x)
    for d in F.near:
        tg, src = F._pairs[d]
        ref[:, tg, :] += x[:, src, :] @ (F.S[d] - F.S_exact[d]).T
    assert rel(diff, ref) < 1e-9
    # storage: the multilevel plan keeps no n x n blocks
    assert P2.info["resident_bytes"] < P1.info["resident_bytes"]
    P1.close()
    P2.close()


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_multilevel_solve_matches_lu(inner):
    import paper_2201_12050_amd as fm
    v, t, lat, k, F, A = _case("sphere80_3x3_L2")
    _, grid, _, nt, levels, ntn = CASES["sphere80_3x3_L2"]
    P = fm.Plan(v, t, grid, lat.pitch, k, nt, near_levels=levels, near_order=ntn)
    dirs = unit_directions(2, 31)
    b = bem.rhs_plane_wave(v, t, lat, k, -1j / k, dirs)
    xl = np.stack([solve.lu_solve(A, b[q]) for q in range(2)])
    xs, info = P.solve(P.incident_plane_wave(dirs), tol=1e-11, inner=inner)
    assert max(i["rel_residual"] for i in info) <= 1e-11
    assert rel(xs.cpu().numpy().reshape(xl.shape), xl) < 1e-8
    P.close()


def test_multilevel_in_a_batch_with_a_dense_plan():
    # grouped launches: an FMPBEM2 plan and an FMPBEM plan solved together equal each alone
    import paper_2201_12050_amd as fm
    v, t, lat, k, F, A = _case("sphere80_3x3_L2")
    _, grid, _, nt, levels, ntn = CASES["sphere80_3x3_L2"]
    P2 = fm.Plan(v, t, grid, lat.pitch, k, nt, near_levels=levels, near_order=ntn)
    P1 = fm.Plan(v, t, (4, 2, 1), lat.pitch, k, nt)
    b2 = P2.incident_plane_wave(unit_directions(3, 5))
    b1 = P1.incident_plane_wave(unit_directions(2, 6))
    for ortho in ("once", "dgks"):
        o = dict(tol=1e-10, inner="fp32", ortho=ortho)
        res = fm.solve_batch([(P2, b2, None, o), (P1, b1, None, o)])
        for P, b, (x, infos) in zip((P2, P1), (b2, b1), res):
            assert max(i["rel_residual"] for i in infos) <= 1e-10
            xa, _ = P.solve(b, **o)
            assert rel(x.cpu().numpy(), xa.cpu().numpy()) < 1e-8
    P1.close()
    P2.close()


def test_multilevel_in_the_engine():
    # serving form: an FMPBEM2 request and a dense-near request in one engine, each equal to its
    # own solve
    import paper_2201_12050_amd as fm
    v, t, lat, k, F, A = _case("sphere80_3x3_L2")
    _, grid, _, nt, levels, ntn = CASES["sphere80_3x3_L2"]
    P2 = fm.Plan(v, t, grid, lat.pitch, k, nt, near_levels=levels, near_order=ntn)
    P1 = fm.Plan(v, t, (4, 2, 1), lat.pitch, k, nt)
    b2 = P2.incident_plane_wave(unit_directions(2, 15))
    b1 = P1.incident_plane_wave(unit_directions(3, 16))
    o = dict(tol=1e-10, inner="fp32", ortho="once")
    E = fm.Engine(hbm_budget_bytes=8 << 30, max_slots=4)
    t2, t1 = E.submit(P2, b2, **o), E.submit(P1, b1, **o)
    done = {}
    for _ in range(100000):
        for tk in (t2, t1):
            if tk not in done:
                r = E.poll(tk)
                if r is not None:
                    done[tk] = r
        if len(done) == 2:
            break
        E.step()
    assert len(done) == 2
    for tk, P, b in ((t2, P2, b2), (t1, P1, b1)):
        x, infos, st = done[tk]
        assert st == 0 and max(i["rel_residual"] for i in infos) <= 1e-10
        xa, _ = P.solve(b, **o)
        assert rel(x.cpu().numpy(), xa.cpu().numpy()) < 1e-8
    E.close()
    P1.close()
    P2.close()


def test_multilevel_noalloc_equals_workspace_entry_point():
    import paper_2201_12050_amd as fm
    v, t, lat, k, F, A = _case("sphere80_3x3_L2")
    _, grid, _, nt, levels, ntn = CASES["sphere80_3x3_L2"]
    P = fm.Plan(v, t, grid, lat.pitch, k, nt, near_levels=levels, near_order=ntn)
    x = torch.from_numpy(random_complex((2, lat.n_cells, t.shape[0]), 91)).cuda()
    for prec, xx in (("fp64", x), ("fp32", x.to(torch.complex64))):
        y_ws = P.matvec(xx, precision=prec)
        y_na = torch.full_like(xx, float("nan"))
        P.matvec_noalloc(xx, y_na, precision=prec)
        assert torch.isfinite(torch.view_as_real(y_na)).all()
        assert rel(y_na.cpu().numpy(), y_ws.cpu().numpy()) < (1e-13 if prec == "fp64" else 1e-6)
    P.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_multilevel_profile_counts_each_application_once(prec):
    # an FMPBEM2 application records its multilevel products as several intervals on two streams
    # (tree stages, P2P blocks, L2P); the stage's count is the number of applications and its time
    # covers every interval, whether the marks are read at once or after later applications
    import paper_2201_12050_amd as fm
    v, t, lat, k, F, A = _case("sphere80_3x3_L2")
    _, grid, _, nt, levels, ntn = CASES["sphere80_3x3_L2"]
    P = fm.Plan(v, t, grid, lat.pitch, k, nt, near_levels=levels, near_order=ntn)
    x = torch.from_numpy(random_complex((1, lat.n_cells, t.shape[0]), 5)).cuda()
    x = x.to(torch.complex64) if prec == "fp32" else x
    ref = P.matvec(x, precision=prec)
    P.profile([f"reduce_{prec}", f"fft_{prec}"])
    for _ in range(3):
        y = P.matvec(x, precision=prec)
    torch.cuda.synchronize()
    first = P.profile_read()
    for _ in range(2):
        y = P.matvec(x, precision=prec)
    second = P.profile_read()
    P.profile([])
    assert first[f"reduce_{prec}"][1] == 3 and second[f"reduce_{prec}"][1] == 5
    assert first[f"fft_{prec}"][1] == 3 and second[f"fft_{prec}"][1] == 5
    assert 0 < first[f"reduce_{prec}"][0] < second[f"reduce_{prec}"][0]
    assert rel(y.cpu().numpy(), ref.cpu().numpy()) < 1e-12
    P.close()


def test_multilevel_task_lists_longer_than_a_wave():
    # a 16x16x8 lattice (27 near offsets) with 3 levels: the M2L stage is not split, and a box
    # interacts with up to 189 source boxes, so the product kernel walks task lists in several
    # batches of 64 descriptors.  Sampled rows against the oracle's FMPBEM2 (computed here).
    import paper_2201_12050_amd as fm
    v, t = icosphere(1, 0.1)
    lat = Lattice((16, 16, 8), (0.3, 0.3, 0.3))
    k = 2 * np.pi * 700 / 343.0
    P = fm.Plan(v, t, lat.grid, lat.pitch, k, 4, near_levels=3, near_order=2)
    assert P.info["near_max_tasks"] > 128
    n = t.shape[0]
    x = random_complex((1, lat.n_cells, n), 2301)
    rng = np.random.default_rng(23011)
    cells = [0, 17, 255, 1000, 1535, 2047]      # corners, an edge and the interior
    dofs = [c * n + int(e) for c in cells for e in rng.integers(0, n, size=3)]
    ref = ml.sampled_apply2(v, t, lat, k, 4, -1j / k, 3, 2, x, dofs)[0]
    xd = torch.from_numpy(x).cuda()
    y64 = P.matvec(xd, precision="fp64").cpu().numpy().reshape(-1)[dofs]
    y32 = P.matvec(xd.to(torch.complex64), precision="fp32").cpu().numpy().reshape(-1)[dofs]
    for y, tol in ((y64, 1e-12), (y32, 1e-5)):
        assert rel(y, ref) < tol   # relative l2 and max-norm
    P.close()
