"""Pins for the singular and near-singular integrals of oracle.bem.

* The split finite-part self term equals an independent contour form of the
  same integral (in-plane divergence theorem):
      FP int_T d2G/dn_x dn_y dA = oint_dT dG/dnu ds + k^2 int_T G dA
  (on a flat element d2G/dn_x dn_y = -d2G/dz2 = Delta_2D G + k^2 G).
* Laplace solid-angle identity: for a closed surface with the normal pointing
  into the scatterer, int_Gamma dG0/dn_y dA = 1/2 at a smooth surface point, so
  every row of (1/2 I + D) at k = 0 sums to 1; with the opposite orientation it
  sums to 0.
"""
import numpy as np
import pytest

from oracle import bem, quadrature
from workloads import icosphere


def contour_self(a, b, c, x, k, qe=256, qa=64):
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n)
    cen = (a + b + c) / 3
    tot = 0.0 + 0.0j
    xs, ws = quadrature.gauss_legendre(qe)
    for p, q in ((a, b), (b, c), (c, a)):
        e = q - p
        L = np.linalg.norm(e)
        nu = np.cross(e, n)
        nu /= np.linalg.norm(nu)
        if np.dot(nu, (p + q) / 2 - cen) < 0:
            nu = -nu
        y = p[None] + ((xs + 1) / 2)[:, None] * e[None]
        r = y - x
        R = np.linalg.norm(r, axis=1)
        dG = np.exp(1j * k * R) / (4 * np.pi) * (1j * k * R - 1) / R ** 2 * (r @ nu) / R
        tot += (dG * ws / 2 * L).sum()
    for p, q in ((a, b), (b, c), (c, a)):
        pts, w = quadrature.duffy_points(x, p, q, qa)
        R = np.linalg.norm(pts - x, axis=-1)
        tot += k * k * (np.exp(1j * k * R) / (4 * np.pi * R) * w).sum()
    return tot


@pytest.mark.parametrize("k", [0.0, 9.159, 18.318, 60.0])
def test_self_term_converges_to_contour_form(k):
    rng = np.random.default_rng(0)
    for _ in range(3):
        a, b, c = rng.normal(size=(3, 3)) * 0.05
        x = (a + b + c) / 3
        ref = contour_self(a, b, c, x, k, qe=512, qa=96)
        assert abs(bem.hypersingular_self(a, b, c, x, k, q=96) - ref) < 1e-11 * abs(ref)


def test_self_term_rule_accuracy_on_mesh_elements():
    # icosphere level-2 elements at up to 2 kHz: the 16x16 rule is accurate to 1e-8
    v, t = icosphere(2, 0.1)
    g = bem.element_geometry(v, t)
    for k in (9.159, 36.6):
        for i in (0, 17, 200):
            a, b, c, x = g["a"][i], g["b"][i], g["c"][i], g["centroid"][i]
            ref = contour_self(a, b, c, x, k)
            assert abs(bem.hypersingular_self(a, b, c, x, k) - ref) < 1e-8 * abs(ref)


def test_fp_closed_form_is_laplace_contour():
    rng = np.random.default_rng(4)
    for _ in range(5):
        a, b, c = rng.normal(size=(3, 3))
        x = (a + b + c) / 3
        assert abs(bem.fp_inv_r3(a, b, c, x) / (4 * np.pi) - contour_self(a, b, c, x, 0.0).real) < 1e-10


def test_equilateral_fp_value():
    # closed form for an equilateral triangle of side s at its centre: each edge is at
    # h = s/(2 sqrt 3) and its ends are seen at +-60 degrees from the foot of the
    # perpendicular, so FP = -3 * (2 sin 60deg) / h = -18 / s.
    s = 0.7
    a = np.array([0.0, 0.0, 0.0]); b = np.array([s, 0.0, 0.0]); c = np.array([s / 2, s * np.sqrt(3) / 2, 0.0])
    x = (a + b + c) / 3
    assert np.isclose(bem.fp_inv_r3(a, b, c, x), -18.0 / s, rtol=1e-14)


@pytest.mark.parametrize("flip", [False, True])
def test_solid_angle_identity(flip):
    v, t = icosphere(2, 0.1)
    if flip:
        t = t[:, [0, 2, 1]]
    g = bem.element_geometry(v, t)
    B = bem.block(g, 0.0, 0.0, np.zeros(3), np.zeros(3), True)
    target = 0.0 if flip else 1.0
    assert np.abs(B.sum(1) - target).max() < 1e-7
