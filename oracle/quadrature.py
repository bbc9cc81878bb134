"""Quadrature rules (oracle; test infrastructure).

The paper leaves the integration scheme to the cited BEM literature (Sec. 2.1,
after eq. (matrixBEM)).  The rule used by both the oracle and the HIP library
is fixed here, so that the two independent implementations produce the same
discrete operator:

* Gauss-Legendre nodes on [-1, 1] computed by Newton's method on P_q.
* Duffy-collapsed product rule on a triangle (a, b, c), collapsed at a:
      y(u, v) = a + u [ (b - a) + v (c - b) ],   u, v in [0, 1],
      dA = |(b - a) x (c - a)| u du dv,
  with q x q Gauss-Legendre points in (u, v).
"""
from __future__ import annotations

import math

import numpy as np


def gauss_legendre(q: int):
    """Nodes (ascending) and weights of the q-point Gauss-Legendre rule on [-1, 1]."""
    if q < 1:
        raise ValueError("q >= 1")
    i = np.arange(q, dtype=np.float64)
    x = np.cos(math.pi * (i + 0.75) / (q + 0.5))
    for _ in range(100):
        p0 = np.ones_like(x)
        p1 = x.copy()
        for j in range(2, q + 1):
            p0, p1 = p1, ((2 * j - 1) * x * p1 - (j - 1) * p0) / j
        if q == 1:
            p0 = np.ones_like(x)
        dp = q * (x * p1 - p0) / (x * x - 1.0)
        dx = p1 / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-15:
            break
    # recompute derivative at converged nodes
    p0 = np.ones_like(x)
    p1 = x.copy()
    for j in range(2, q + 1):
        p0, p1 = p1, ((2 * j - 1) * x * p1 - (j - 1) * p0) / j
    if q == 1:
        p0 = np.ones_like(x)
    dp = q * (x * p1 - p0) / (x * x - 1.0)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    order = np.argsort(x)
    return x[order], w[order]


def unit_duffy(q: int):
    """(u, v, w) of the q x q collapsed rule on the reference square, where the
    weight already contains the Duffy Jacobian factor u and the 1/4 of the two
    [-1,1] -> [0,1] maps; multiply by |(b-a)x(c-a)| for a physical triangle."""
    x, w = gauss_legendre(q)
    t = 0.5 * (x + 1.0)
    u = np.repeat(t, q)
    v = np.tile(t, q)
    ww = np.repeat(w, q) * np.tile(w, q) * 0.25 * u
    return u, v, ww


def duffy_points(a, b, c, q: int):
    """Quadrature points [.., q*q, 3] and weights [.., q*q] on triangles (a, b, c)
    (arrays [..., 3]) collapsed at vertex a."""
    u, v, w = unit_duffy(q)
    a = np.asarray(a)[..., None, :]
    b = np.asarray(b)[..., None, :]
    c = np.asarray(c)[..., None, :]
    pts = a + u[:, None] * ((b - a) + v[:, None] * (c - b))
    jac = np.linalg.norm(np.cross(b - a, c - a), axis=-1)  # [..., 1]
    return pts, w * jac
