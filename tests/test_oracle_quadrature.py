"""Pins for oracle.quadrature: library routine and exact polynomial integration."""
import numpy as np
import pytest

from oracle.quadrature import gauss_legendre, duffy_points


@pytest.mark.parametrize("q", [1, 2, 3, 4, 7, 8, 16, 24])
def test_gauss_legendre_matches_numpy(q):
    x, w = gauss_legendre(q)
    xr, wr = np.polynomial.legendre.leggauss(q)
    assert np.allclose(x, xr, atol=1e-14, rtol=0)
    assert np.allclose(w, wr, atol=1e-14, rtol=0)


@pytest.mark.parametrize("q", [2, 4, 8, 16])
def test_gauss_legendre_exact_degree(q):
    x, w = gauss_legendre(q)
    for deg in range(2 * q):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs((w * x ** deg).sum() - exact) < 1e-13


def _tri_moments(a, b, c):
    """Closed forms: area, first moments and second moments of a triangle."""
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a))
    s = a + b + c
    m1 = area * s / 3.0
    m2 = area / 12.0 * (np.outer(a, a) + np.outer(b, b) + np.outer(c, c) + np.outer(s, s))
    return area, m1, m2


@pytest.mark.parametrize("q", [2, 4, 8, 16])
def test_duffy_rule_polynomials(q):
    rng = np.random.default_rng(3)
    for _ in range(5):
        a, b, c = rng.normal(size=(3, 3))
        pts, w = duffy_points(a, b, c, q)
        area, m1, m2 = _tri_moments(a, b, c)
        assert abs(w.sum() - area) < 1e-13 * max(1, area)
        assert np.allclose((w[:, None] * pts).sum(0), m1, atol=1e-12)
        assert np.allclose(np.einsum("q,qi,qj->ij", w, pts, pts), m2, atol=1e-12)
