"""Pins for oracle.kernels: central finite differences of G and the Laplace limit."""
import numpy as np
import pytest

from oracle import kernels


def _setup(seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=3)
    y = x + rng.normal(size=3) * 0.3
    nx = rng.normal(size=3); nx /= np.linalg.norm(nx)
    ny = rng.normal(size=3); ny /= np.linalg.norm(ny)
    return x, y, nx, ny


@pytest.mark.parametrize("k", [0.5, 9.159, 18.318, 40.0])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_normal_derivatives_finite_differences(k, seed):
    x, y, nx, ny = _setup(seed)
    R = np.linalg.norm(x - y)
    h = 1e-3 * R

    def d(f):  # fourth-order central difference along s
        return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)

    fd_ny = d(lambda s: kernels.green(x, y + s * ny, k))
    fd_nx = d(lambda s: kernels.green(x + s * nx, y, k))
    fd_nxny = d(lambda s: kernels.dgreen_dny(x + s * nx, y, ny, k))
    assert abs(kernels.dgreen_dny(x, y, ny, k) - fd_ny) <= 1e-7 * abs(fd_ny) + 1e-9
    assert abs(kernels.dgreen_dnx(x, y, nx, k) - fd_nx) <= 1e-7 * abs(fd_nx) + 1e-9
    assert abs(kernels.d2green_dnxdny(x, y, nx, ny, k) - fd_nxny) <= 1e-6 * abs(fd_nxny) + 1e-9


def test_laplace_limit():
    x, y, nx, ny = _setup(5)
    r = x - y
    R = np.linalg.norm(r)
    k = 1e-9
    assert np.isclose(kernels.green(x, y, k), 1 / (4 * np.pi * R), rtol=1e-12)
    assert np.isclose(kernels.dgreen_dny(x, y, ny, k), (r @ ny) / (4 * np.pi * R ** 3), rtol=1e-12)
    lap = (nx @ ny) / (4 * np.pi * R ** 3) - 3 * (r @ nx) * (r @ ny) / (4 * np.pi * R ** 5)
    assert np.isclose(kernels.d2green_dnxdny(x, y, nx, ny, k), lap, rtol=1e-9)


def test_bm_kernel_is_combination():
    x, y, nx, ny = _setup(7)
    k, a = 3.0, -1j / 3.0
    ref = kernels.dgreen_dny(x, y, ny, k) + a * kernels.d2green_dnxdny(x, y, nx, ny, k)
    assert np.isclose(kernels.bm_kernel(x, y, nx, ny, k, a), ref, rtol=1e-15)
    assert kernels.bm_kernel(x, y, nx, ny, k, 0.0) == kernels.dgreen_dny(x, y, ny, k)
