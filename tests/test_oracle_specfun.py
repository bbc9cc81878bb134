"""Pins for oracle.specfun: library routines, closed forms and identities."""
import math

import numpy as np
import pytest
from scipy import special
from sympy.physics.wigner import wigner_3j as sympy_3j

from oracle import specfun, fmm


def test_wigner3j_matches_sympy_sample():
    rng = np.random.default_rng(11)
    for _ in range(200):
        j1, j2 = rng.integers(0, 9, size=2)
        j3 = rng.integers(abs(j1 - j2), j1 + j2 + 1)
        m1 = rng.integers(-j1, j1 + 1)
        m2 = rng.integers(-j2, j2 + 1)
        m3 = -m1 - m2
        ref = float(sympy_3j(int(j1), int(j2), int(j3), int(m1), int(m2), int(m3)))
        assert abs(specfun.wigner3j(int(j1), int(j2), int(j3), int(m1), int(m2), int(m3)) - ref) < 1e-14


def test_wigner3j_zero_m_closed_form():
    # (j1 j2 j3; 0 0 0) = (-1)^g sqrt[(2g-2j1)!(2g-2j2)!(2g-2j3)!/(2g+1)!] g!/((g-j1)!(g-j2)!(g-j3)!)
    # for J = j1+j2+j3 = 2g even, and 0 for J odd.
    f = math.factorial
    for j1 in range(0, 12):
        for j2 in range(0, 12):
            for j3 in range(abs(j1 - j2), j1 + j2 + 1):
                J = j1 + j2 + j3
                if J % 2:
                    ref = 0.0
                else:
                    g = J // 2
                    ref = (-1) ** g * math.sqrt(f(2 * g - 2 * j1) * f(2 * g - 2 * j2) * f(2 * g - 2 * j3) / f(2 * g + 1)) \
                        * f(g) / (f(g - j1) * f(g - j2) * f(g - j3))
                assert abs(specfun.wigner3j(j1, j2, j3, 0, 0, 0) - ref) < 1e-14


def test_wigner3j_special_and_orthogonality():
    for j in range(0, 10):
        for m in range(-j, j + 1):
            assert abs(specfun.wigner3j(j, j, 0, m, -m, 0) - (-1) ** (j - m) / math.sqrt(2 * j + 1)) < 1e-15
    j1, j2 = 4, 3
    for j3 in range(1, 8):
        for j3b in range(1, 8):
            for m3 in range(-min(j3, j3b), min(j3, j3b) + 1):
                s = sum(specfun.wigner3j(j1, j2, j3, m1, -m1 - m3, m3) * specfun.wigner3j(j1, j2, j3b, m1, -m1 - m3, m3)
                        for m1 in range(-j1, j1 + 1) if abs(m1 + m3) <= j2)
                ref = (1.0 / (2 * j3 + 1)) if j3 == j3b else 0.0
                assert abs(s - ref) < 1e-14


def test_spherical_bessel_closed_forms():
    x = np.linspace(0.3, 20.0, 50)
    assert np.allclose(specfun.sph_j(0, x), np.sin(x) / x, rtol=1e-13)
    assert np.allclose(specfun.sph_j(1, x), np.sin(x) / x ** 2 - np.cos(x) / x, rtol=1e-12, atol=1e-15)
    assert np.allclose(specfun.sph_h(0, x), -1j * np.exp(1j * x) / x, rtol=1e-13)
    assert np.allclose(specfun.sph_h(1, x), -np.exp(1j * x) * (x + 1j) / x ** 2, rtol=1e-12)


def test_harmonics_low_order_closed_forms():
    rng = np.random.default_rng(2)
    ct = rng.uniform(-1, 1, 20)
    phi = rng.uniform(-np.pi, np.pi, 20)
    st = np.sqrt(1 - ct ** 2)
    Y = specfun.harmonics(ct, phi, 2)
    assert np.allclose(Y[:, specfun.idx(0, 0)], 1.0)
    assert np.allclose(Y[:, specfun.idx(1, 0)], ct)
    assert np.allclose(Y[:, specfun.idx(1, 1)], -st * np.exp(1j * phi) / math.sqrt(2))
    assert np.allclose(Y[:, specfun.idx(1, -1)], st * np.exp(-1j * phi) / math.sqrt(2))
    assert np.allclose(Y[:, specfun.idx(2, 0)], 0.5 * (3 * ct ** 2 - 1))
    assert np.allclose(Y[:, specfun.idx(2, 2)], math.sqrt(1 / 24) * 3 * st ** 2 * np.exp(2j * phi))


@pytest.mark.parametrize("nmax", [6, 14])
def test_harmonics_addition_theorem(nmax):
    rng = np.random.default_rng(5)
    a = rng.normal(size=(10, 3)); a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = rng.normal(size=(10, 3)); b /= np.linalg.norm(b, axis=1, keepdims=True)
    Ya = specfun.harmonics(a[:, 2], np.arctan2(a[:, 1], a[:, 0]), nmax)
    Yb = specfun.harmonics(b[:, 2], np.arctan2(b[:, 1], b[:, 0]), nmax)
    cg = (a * b).sum(1)
    for n in range(nmax + 1):
        s = (Ya[:, n * n:(n + 1) ** 2] * np.conj(Yb[:, n * n:(n + 1) ** 2])).sum(1)
        assert np.allclose(s, special.eval_legendre(n, cg), atol=1e-12)


def test_regular_gradient_finite_differences():
    rng = np.random.default_rng(8)
    k = 18.318
    v = rng.normal(size=(6, 3)) * 0.1
    g = fmm.grad_conj_regular(v, k, 8)
    h = 1e-4
    for i in range(3):
        e = np.zeros(3); e[i] = h
        fd = (-np.conj(fmm.regular(v + 2 * e, k, 8)) + 8 * np.conj(fmm.regular(v + e, k, 8))
              - 8 * np.conj(fmm.regular(v - e, k, 8)) + np.conj(fmm.regular(v - 2 * e, k, 8))) / (12 * h)
        assert np.allclose(g[..., i], fd, atol=1e-9, rtol=1e-7)
