"""Special functions for the multipole expansion (oracle; test infrastructure).

* j_n, y_n, h_n = j_n + i y_n: SciPy's spherical Bessel functions.
* Associated Legendre P_n^m WITHOUT the Condon-Shortley phase, from SciPy's
  ``lpmv`` (which includes it): P_n^m = (-1)^m lpmv(m, n, .).
* Harmonics, the reading of Sec. 3.1 (the paper only cites the convention):
      Y_n^m(theta, phi) = (-1)^m sqrt((n-m)!/(n+m)!) P_n^m(cos theta) e^{i m phi},  m >= 0
      Y_n^{-m} = (-1)^m conj(Y_n^m)
  so that sum_m Y_n^m(a) conj(Y_n^m(b)) = P_n(a.b).
* Wigner 3j symbols by Racah's formula in exact integer arithmetic.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import numpy as np
from scipy import special


def sph_j(n, x):
    return special.spherical_jn(n, x)


def sph_jd(n, x):
    return special.spherical_jn(n, x, derivative=True)


def sph_h(n, x):
    return special.spherical_jn(n, x) + 1j * special.spherical_yn(n, x)


def sph_hd(n, x):
    return special.spherical_jn(n, x, derivative=True) + 1j * special.spherical_yn(n, x, derivative=True)


def legendre_nocs(n, m, x):
    """P_n^m(x) without the Condon-Shortley phase (m >= 0); 0 when m > n."""
    if m > n:
        return np.zeros_like(np.asarray(x, dtype=np.float64))
    return (-1.0) ** m * special.lpmv(m, n, x)


def idx(n: int, m: int) -> int:
    """Position of (n, m) in a coefficient vector of length (n_t+1)^2."""
    return n * n + n + m


def spherical_coords(v):
    v = np.asarray(v, dtype=np.float64)
    r = np.linalg.norm(v, axis=-1)
    rr = np.where(r > 0, r, 1.0)
    ct = np.clip(v[..., 2] / rr, -1.0, 1.0)
    phi = np.arctan2(v[..., 1], v[..., 0])
    return r, ct, phi


def harmonics(ct, phi, nmax: int, with_dtheta: bool = False):
    """Y_n^m(theta, phi) for all n <= nmax, |m| <= n, at cos(theta) = ct.

    Returns Y [..., (nmax+1)^2] (and dY/dtheta of the same shape)."""
    ct = np.asarray(ct, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    shape = ct.shape + ((nmax + 1) ** 2,)
    Y = np.zeros(shape, dtype=np.complex128)
    dY = np.zeros(shape, dtype=np.complex128) if with_dtheta else None
    for n in range(nmax + 1):
        for m in range(0, n + 1):
            norm = (-1.0) ** m * math.sqrt(math.factorial(n - m) / math.factorial(n + m))
            P = legendre_nocs(n, m, ct)
            e = np.exp(1j * m * phi)
            y = norm * P * e
            Y[..., idx(n, m)] = y
            if m > 0:
                Y[..., idx(n, -m)] = (-1.0) ** m * np.conj(y)
            if with_dtheta:
                # (x^2 - 1) dP_n^m/dx = n x P_n^m - (n + m) P_{n-1}^m, x = cos(theta)
                Pm1 = legendre_nocs(n - 1, m, ct) if n >= 1 else np.zeros_like(ct)
                dP = (n * ct * P - (n + m) * Pm1) / np.where(st > 0, st, np.inf)
                dy = norm * dP * e
                dY[..., idx(n, m)] = dy
                if m > 0:
                    dY[..., idx(n, -m)] = (-1.0) ** m * np.conj(dy)
    return (Y, dY) if with_dtheta else Y


@lru_cache(maxsize=None)
def wigner3j(j1: int, j2: int, j3: int, m1: int, m2: int, m3: int) -> float:
    """Wigner 3j symbol (j1 j2 j3; m1 m2 m3) for integer arguments, Racah's formula."""
    if m1 + m2 + m3 != 0:
        return 0.0
    if j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    f = math.factorial
    tri = Fraction(f(j1 + j2 - j3) * f(j1 - j2 + j3) * f(-j1 + j2 + j3), f(j1 + j2 + j3 + 1))
    pref = (f(j1 + m1) * f(j1 - m1) * f(j2 + m2) * f(j2 - m2) * f(j3 + m3) * f(j3 - m3))
    tmin = max(0, j2 - j3 - m1, j1 - j3 + m2)
    tmax = min(j1 + j2 - j3, j1 - m1, j2 + m2)
    s = Fraction(0)
    for t in range(tmin, tmax + 1):
        den = (f(t) * f(j3 - j2 + t + m1) * f(j3 - j1 + t - m2) * f(j1 + j2 - j3 - t)
               * f(j1 - t - m1) * f(j2 - t + m2))
        s += Fraction((-1) ** t, den)
    if s == 0:
        return 0.0
    sq = tri * pref * s * s
    sign = (1 if s > 0 else -1) * (-1) ** ((j1 - j2 - m3) % 2)
    return sign * math.sqrt(float(sq))
