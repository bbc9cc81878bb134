"""Pins for the half-space oracle (eq. (green3dHalf), Sec. 2.3, Sec. 3.4, eq. (greenFMMhalfspace)).

The method of images is the independent reference: a rigid (R_p = 1) or soft (R_p = -1)
plane z = z_g above a sphere at the origin is the full-space problem of the sphere and
its mirror image (a 1 x 1 x 2 lattice with pitch 2 z_g) under the symmetric or
antisymmetric excitation, so the half-space solution equals the full-space one on the
lower cell.  A wrong sign of the mirrored normal, a missing image term or a wrong image
of the incident field fails it.  The multipole form converges to the dense one in n_t
(a wrong reflection factor D_z leaves an O(1) error)."""
import numpy as np
import pytest

from oracle import bem, halfspace as hs, operator as op, solve
from workloads import Lattice, icosphere

ZG = 0.15
LAT1 = Lattice((1, 1, 1), (0.3, 0.3, 0.3))
LAT2 = Lattice((1, 1, 2), (0.3, 0.3, 0.3))   # the sphere and its image at z = 2 z_g


@pytest.mark.parametrize("formulation", ["bm", "cbie"])
@pytest.mark.parametrize("rp", [1.0, -1.0])
def test_method_of_images_plane_wave(formulation, rp):
    v, t = icosphere(1, 0.1)
    k = 2 * np.pi * 600.0 / 343.0
    a = bem.default_alpha(k, formulation)
    d = [0.6, 0.0, 0.8]
    xh = solve.lu_solve(hs.dense_exact(v, t, LAT1, k, a, ZG, rp), hs.rhs_plane_wave(v, t, LAT1, k, a, [d], ZG, rp)[0])
    # full space: the incident wave and its image, on both spheres
    dm = [0.6, 0.0, -0.8]
    b = (bem.rhs_plane_wave(v, t, LAT2, k, a, [d])[0] +
         bem.rhs_plane_wave(v, t, LAT2, k, a, [dm], rp * np.exp(2j * k * ZG * d[2]))[0])
    xf = solve.lu_solve(bem.dense_exact(v, t, LAT2, k, a), b)
    n = t.shape[0]
    assert np.linalg.norm(xh - xf[:n]) < 1e-8 * np.linalg.norm(xf[:n])


def test_method_of_images_point_source_and_field():
    v, t = icosphere(1, 0.1)
    k = 2 * np.pi * 450.0 / 343.0
    a = bem.default_alpha(k, "bm")
    src = np.array([[0.4, -0.3, -0.2]])
    xh = solve.lu_solve(hs.dense_exact(v, t, LAT1, k, a, ZG, 1.0),
                        hs.rhs_point_source(v, t, LAT1, k, a, src, ZG, 1.0)[0])
    img = src.copy()
    img[:, 2] = 2 * ZG - img[:, 2]
    b = bem.rhs_point_source(v, t, LAT2, k, a, src)[0] + bem.rhs_point_source(v, t, LAT2, k, a, img)[0]
    xf = solve.lu_solve(bem.dense_exact(v, t, LAT2, k, a), b)
    n = t.shape[0]
    assert np.linalg.norm(xh - xf[:n]) < 1e-8 * np.linalg.norm(xf[:n])
    # the pressure below the plane: half-space representation vs the full-space one of both spheres
    pts = np.array([[0.5, 0.2, -0.3], [-0.2, 0.6, 0.05], [0.0, 0.0, -0.8]])
    ph = hs.field(v, t, LAT1, k, pts, xh, ZG, 1.0, hs.incident_point_source_at(pts, k, src, ZG, 1.0))
    pf = bem.field(v, t, LAT2, k, pts, xf,
                   bem.incident_point_source_at(pts, k, src) + bem.incident_point_source_at(pts, k, img))
    assert np.linalg.norm(ph - pf) < 1e-8 * np.linalg.norm(pf)


def test_zero_reflection_is_full_space():
    v, t = icosphere(1, 0.1)
    lat = Lattice((4, 3, 1), (0.3, 0.3, 0.3))
    k = 2 * np.pi * 600.0 / 343.0
    F = op.FMPBEM(v, t, lat, k, 6, -1j / k)
    H = hs.FMPBEMHalfSpace(v, t, lat, k, 6, -1j / k, ZG, 0.0)
    x = np.random.default_rng(0).normal(size=(2, 12, 80)) + 0j
    assert np.array_equal(F.matvec(x), H.matvec(x))


def test_multipole_image_converges_to_dense():
    # a complex reflection coefficient, image blocks near (|2 z_g| < 2 pitch) and far
    v, t = icosphere(1, 0.1)
    lat = Lattice((4, 3, 1), (0.3, 0.3, 0.3))
    k = 2 * np.pi * 600.0 / 343.0
    A1 = hs.dense_exact(v, t, lat, k, -1j / k, ZG, 0.7 - 0.3j)
    errs = []
    for nt in (4, 8):
        H = hs.FMPBEMHalfSpace(v, t, lat, k, nt, -1j / k, ZG, 0.7 - 0.3j)
        assert len(H.img_near) == 9 and len(H.img_far) == 26
        errs.append(np.linalg.norm(H.dense() - A1) / np.linalg.norm(A1))
    assert errs[0] < 1e-4 and errs[1] < errs[0] / 1000


def test_image_entirely_far():
    # a plane far below: no image block is near, every image block goes through U K^ D_z V
    v, t = icosphere(1, 0.1)
    lat = Lattice((3, 2, 1), (0.3, 0.3, 0.3))
    k = 2 * np.pi * 500.0 / 343.0
    H = hs.FMPBEMHalfSpace(v, t, lat, k, 8, -1j / k, -0.45, 1.0)
    assert H.img_near == [] and len(H.img_far) == 15
    A1 = hs.dense_exact(v, t, lat, k, -1j / k, -0.45, 1.0)
    assert np.linalg.norm(H.dense() - A1) < 1e-6 * np.linalg.norm(A1)


def test_surface_must_not_cross_plane():
    v, t = icosphere(1, 0.1)
    with pytest.raises(ValueError):
        hs.dense_exact(v, t, LAT1, 3.0, 0.0, 0.05, 1.0)
    with pytest.raises(ValueError):
        hs.FMPBEMHalfSpace(v, t, Lattice((2, 2, 2), (0.3, 0.3, 0.3)), 3.0, 4, 0.0, 0.2, 1.0)


@pytest.mark.parametrize("rp", [1.0, -1.0])
def test_method_of_images_periodic_normal_to_plane(rp):
    # second case of Sec. 3.4: two spheres stacked along z (pitch 0.3) above the plane z = -0.15;
    # with their two images this is a 1 x 1 x 4 full-space lattice, shifted up by 0.6 so that its
    # cells sit at z = 0, 0.3 (images) and 0.6, 0.9 (the originals)
    v, t = icosphere(1, 0.1)
    k = 2 * np.pi * 500.0 / 343.0
    a = bem.default_alpha(k, "bm")
    zg = -0.15
    lat = Lattice((1, 1, 2), (0.3, 0.3, 0.3))
    src = np.array([[0.5, -0.4, 0.2]])
    xh = solve.lu_solve(hs.dense_exact(v, t, lat, k, a, zg, rp), hs.rhs_point_source(v, t, lat, k, a, src, zg, rp)[0])
    lat4 = Lattice((1, 1, 4), (0.3, 0.3, 0.3))
    up = np.array([[0.0, 0.0, 0.6]])
    img = src.copy()
    img[:, 2] = 2 * zg - img[:, 2]
    b = (bem.rhs_point_source(v, t, lat4, k, a, src + up)[0] +
         bem.rhs_point_source(v, t, lat4, k, a, img + up, rp)[0])
    xf = solve.lu_solve(bem.dense_exact(v, t, lat4, k, a), b)
    n = t.shape[0]
    assert np.linalg.norm(xh - xf[2 * n:]) < 1e-8 * np.linalg.norm(xf[2 * n:])


def test_multipole_image_converges_to_dense_periodic_normal_to_plane():
    # 3 x 1 x 3 lattice standing on the plane: image blocks near for the lowest layer only
    v, t = icosphere(1, 0.1)
    lat = Lattice((3, 1, 3), (0.3, 0.3, 0.3))
    k = 2 * np.pi * 500.0 / 343.0
    zg = -0.15
    A1 = hs.dense_exact(v, t, lat, k, -1j / k, zg, 0.8 + 0.2j)
    errs = []
    for nt in (4, 8):
        H = hs.FMPBEMHalfSpace(v, t, lat, k, nt, -1j / k, zg, 0.8 + 0.2j)
        assert sorted({o[2] for o in H.img_near}) == [0]
        errs.append(np.linalg.norm(H.dense() - A1) / np.linalg.norm(A1))
    assert errs[0] < 1e-4 and errs[1] < errs[0] / 100
