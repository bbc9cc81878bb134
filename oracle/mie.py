"""Mie series for plane-wave scattering by one rigid sphere (oracle; analytic pin).

Incident p_inc = e^{ik d.x}, time convention e^{-i w t} (Sec. 2.1).  Expanding
p_inc = sum_n i^n (2n+1) j_n(kr) P_n(cos t) and imposing dp/dr = 0 at r = a gives
the total surface pressure

    p(a, t) = sum_n i^n (2n+1) [j_n(ka) - j_n'(ka) h_n(ka) / h_n'(ka)] P_n(cos t)
            = sum_n i^{n+1} (2n+1) P_n(cos t) / ((ka)^2 h_n'(ka)),

the second form by the Wronskian j_n y_n' - j_n' y_n = 1/x^2.  Off the surface, at
r >= a, the total pressure is

    p(r, t) = sum_n i^n (2n+1) [j_n(kr) - j_n'(ka) h_n(kr) / h_n'(ka)] P_n(cos t).

Point source (monopole p_inc = A e^{ikR}/R, R = |x - s|, Sec. 4.2) at distance r_s > a
from the centre: the addition theorem gives, for r < r_s,
p_inc = A ik sum_n (2n+1) j_n(kr) h_n(k r_s) P_n(cos g), g the angle between x and s.
The rigid boundary condition and the same Wronskian reduce the surface pressure to

    p(a, g) = -A sum_n (2n+1) h_n(k r_s) P_n(cos g) / (k a^2 h_n'(ka)).
"""
from __future__ import annotations

import numpy as np
from scipy import special

from .specfun import sph_h, sph_hd, sph_j, sph_jd


def rigid_sphere_surface_pressure(points, radius, k, direction=(1.0, 0.0, 0.0), n_terms=None):
    pts = np.asarray(points, dtype=np.float64)
    d = np.asarray(direction, dtype=np.float64)
    ct = (pts @ d) / np.linalg.norm(pts, axis=1)
    ka = k * radius
    N = int(ka + 30) if n_terms is None else n_terms
    out = np.zeros(pts.shape[0], dtype=np.complex128)
    for n in range(N + 1):
        out += (1j ** ((n + 1) % 4)) * (2 * n + 1) * special.eval_legendre(n, ct) / (ka * ka * sph_hd(n, ka))
    return out


def rigid_sphere_total_field(points, radius, k, direction=(1.0, 0.0, 0.0), n_terms=None):
    """Total pressure (incident + scattered) at points with |x| >= radius."""
    pts = np.asarray(points, dtype=np.float64)
    d = np.asarray(direction, dtype=np.float64)
    r = np.linalg.norm(pts, axis=1)
    ct = (pts @ d) / r
    ka = k * radius
    N = int(k * r.max() + 30) if n_terms is None else n_terms
    out = np.zeros(pts.shape[0], dtype=np.complex128)
    for n in range(N + 1):
        radial = sph_j(n, k * r) - sph_jd(n, ka) * sph_h(n, k * r) / sph_hd(n, ka)
        out += (1j ** (n % 4)) * (2 * n + 1) * radial * special.eval_legendre(n, ct)
    return out


def rigid_sphere_point_source_surface_pressure(points, radius, k, source, amplitude=1.0, n_terms=None):
    """Total surface pressure of a rigid sphere (centre at the origin) under a monopole at
    ``source`` (|source| > radius), series of the module docstring."""
    pts = np.asarray(points, dtype=np.float64)
    s = np.asarray(source, dtype=np.float64)
    rs = np.linalg.norm(s)
    if rs <= radius:
        raise ValueError("source inside the sphere")
    cg = (pts @ s) / (np.linalg.norm(pts, axis=1) * rs)
    ka = k * radius
    # beyond n ~ ka the terms fall super-geometrically while n < k r_s (h_n'(ka) grows like
    # (2n)!/(ka)^n), and like (a / r_s)^n beyond k r_s
    N = int(ka + 30 + 40 * radius / (rs - radius)) if n_terms is None else n_terms
    out = np.zeros(pts.shape[0], dtype=np.complex128)
    for n in range(N + 1):
        out -= (2 * n + 1) * sph_h(n, k * rs) * special.eval_legendre(n, cg) / (k * radius * radius * sph_hd(n, ka))
    return amplitude * out
