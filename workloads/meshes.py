"""Unit-cell surface meshes in cell-local coordinates (cell centre at the origin).

Orientation convention (Section 2.1 of the paper: the normal points out of the
acoustic domain): for every triangle (v0, v1, v2) the vector
(v1 - v0) x (v2 - v0) points *into* the rigid scatterer, i.e. out of the fluid.
"""
from __future__ import annotations

import numpy as np


def _icosahedron():
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    raw = []
    for a in (-1.0, 1.0):
        for b in (-phi, phi):
            raw.append((0.0, a, b))
            raw.append((a, b, 0.0))
            raw.append((b, 0.0, a))
    v = np.array(raw, dtype=np.float64)
    # edges of the icosahedron are exactly the vertex pairs at distance 2
    d2 = ((v[:, None, :] - v[None, :, :]) ** 2).sum(-1)
    adj = np.abs(d2 - 4.0) < 1e-9
    faces = []
    n = len(v)
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    assert len(faces) == 20
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, np.array(faces, dtype=np.int64)


def _orient_inward(v, f):
    """Flip triangles whose (v1-v0)x(v2-v0) points away from the origin."""
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    nrm = np.cross(b - a, c - a)
    cen = (a + b + c) / 3.0
    flip = (nrm * cen).sum(1) > 0.0
    f = f.copy()
    f[flip, 1], f[flip, 2] = f[flip, 2].copy(), f[flip, 1].copy()
    return f


def icosphere(level: int, radius: float = 1.0):
    """Geodesic sphere: the icosahedron with each face split into 4, ``level`` times.

    Returns (vertices [nv,3] float64, triangles [20*4**level, 3] int32), with
    every vertex on the sphere of the given radius and inward-pointing normals.
    """
    if level < 0:
        raise ValueError("level must be >= 0")
    v, f = _icosahedron()
    f = _orient_inward(v, f)
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(i, j):
            key = (i, j) if i < j else (j, i)
            if key in cache:
                return cache[key]
            p = (np.asarray(verts[i]) + np.asarray(verts[j])) * 0.5
            p /= np.linalg.norm(p)
            verts.append(tuple(p))
            cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        f = np.array(nf, dtype=np.int64)
    v = np.array(verts, dtype=np.float64) * radius
    return v, f.astype(np.int32)


def tube_segment(radius: float, height: float, n_around: int = 32, n_rings: int = 3):
    """Open cylindrical tube segment (no caps), axis along z, centred at the origin.

    ``n_around`` x ``n_rings`` quads, each split into two triangles, so
    2 * n_around * n_rings triangles.  Normals point towards the axis, i.e. into
    the (solid) cylinder that a stack of such segments forms.
    """
    phis = 2.0 * np.pi * np.arange(n_around) / n_around
    zs = -0.5 * height + height * np.arange(n_rings + 1) / n_rings
    verts = np.array([(radius * np.cos(p), radius * np.sin(p), z) for z in zs for p in phis])
    tris = []
    for j in range(n_rings):
        for i in range(n_around):
            a = j * n_around + i
            b = j * n_around + (i + 1) % n_around
            c = (j + 1) * n_around + (i + 1) % n_around
            d = (j + 1) * n_around + i
            tris += [(a, b, c), (a, c, d)]
    f = np.array(tris, dtype=np.int64)
    # orient towards the axis
    v0, v1, v2 = verts[f[:, 0]], verts[f[:, 1]], verts[f[:, 2]]
    nrm = np.cross(v1 - v0, v2 - v0)
    radial = (v0 + v1 + v2) / 3.0
    radial[:, 2] = 0.0
    flip = (nrm * radial).sum(1) > 0.0
    f[flip, 1], f[flip, 2] = f[flip, 2].copy(), f[flip, 1].copy()
    return verts, f.astype(np.int32)


def mesh_is_closed(triangles) -> bool:
    """True when every undirected edge is shared by exactly two triangles, used
    once in each direction (a closed, consistently oriented surface)."""
    directed = {}
    for t in np.asarray(triangles):
        for i in range(3):
            e = (int(t[i]), int(t[(i + 1) % 3]))
            directed[e] = directed.get(e, 0) + 1
    for (a, b), cnt in directed.items():
        if cnt != 1 or directed.get((b, a), 0) != 1:
            return False
    return True
