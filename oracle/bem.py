"""Collocation BEM with flat constant triangles (oracle; test infrastructure).

Discretisation of the Burton-Miller equation (Sec. 2.1, eq. (bm)) for a rigid
surface (dp/dn = 0, so the single-layer terms and the admittance term of
eq. (matrixBEM) drop out):

    A[i, j] = 1/2 delta_ij + int_{Delta_j} [ dG/dn_y + alpha d2G/dn_x dn_y ](x_i, y) dA(y)
    b[i]    = p_inc(x_i) + alpha dp_inc/dn(x_i)

with collocation at element centroids x_i, alpha = -i/k (Sec. 2.1, after
eq. (bm)); the CBIE (eq. (cbie)) is the case alpha = 0, c = 1/2.  The normal
points out of the fluid, into the scatterer (Sec. 2.1).

Quadrature (the paper defers it to the literature; this is the reading both
implementations follow):
  * non-self pairs: Duffy rule collapsed at the first vertex, q x q points with
    q = 16 if |x - centroid_j| < L_j, q = 8 if < 3 L_j, else q = 4, where L_j is
    the longest edge of element j;
  * self pairs: dG/dn_y vanishes on a flat element (r.n_y = 0); the
    hypersingular part is the Hadamard finite part of E(1-ikR)/R^3, split into
    (1/4pi) FP int R^-3 dA, in closed form, plus
    (1/4pi) int [e^{ikR}(1-ikR) - 1] R^-3 dA, a weakly singular remainder
    integrated with a 16 x 16 Duffy rule on each of the three sub-triangles
    (x, v_a, v_b) collapsed at x.

Post-processing (Sec. 2.1, eq. (cbie) with c = 1; eq. (insertionloss)): the pressure
at points of the fluid is the incident field minus the double-layer potential of the
surface pressure, integrated with the same non-self Duffy rule (the paper does not
state a field quadrature; points must lie in the fluid, off the surface).
"""
from __future__ import annotations

import numpy as np

from . import kernels
from .quadrature import duffy_points

FOUR_PI = 4.0 * np.pi


def default_alpha(k: float, formulation: str) -> complex:
    """Burton-Miller coupling -i/k (Sec. 2.1, after eq. (bm)); 0 for the CBIE."""
    if formulation == "cbie":
        return 0.0
    if formulation == "bm":
        return -1j / k
    raise ValueError(formulation)


def element_geometry(vertices, triangles):
    v = np.asarray(vertices, dtype=np.float64)
    t = np.asarray(triangles)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    cr = np.cross(b - a, c - a)
    two_area = np.linalg.norm(cr, axis=1)
    if np.any(two_area <= 0):
        raise ValueError("degenerate triangle")
    longest = np.maximum(np.maximum(np.linalg.norm(b - a, axis=1), np.linalg.norm(c - b, axis=1)),
                         np.linalg.norm(a - c, axis=1))
    return dict(a=a, b=b, c=c, centroid=(a + b + c) / 3.0, normal=cr / two_area[:, None],
                area=0.5 * two_area, longest=longest)


def rule_order(dist, longest):
    """Points per direction of the non-self Duffy rule (see module docstring)."""
    return np.where(dist < longest, 16, np.where(dist < 3.0 * longest, 8, 4))


def fp_inv_r3(a, b, c, x):
    """Hadamard finite part of int_T R^-3 dA over the flat triangle T = (a, b, c)
    for x in its interior: -sum_edges (sin t2 - sin t1) / h, angles measured from
    the foot of the perpendicular from x onto each edge."""
    total = 0.0
    for p, q in ((a, b), (b, c), (c, a)):
        e = q - p
        eh = e / np.linalg.norm(e)
        tp = np.dot(p - x, eh)
        tq = np.dot(q - x, eh)
        h = np.linalg.norm((p - x) - tp * eh)
        total -= (tq / np.linalg.norm(q - x) - tp / np.linalg.norm(p - x)) / h
    return total


def hypersingular_self(a, b, c, x, k, q: int = 16):
    """Finite-part value of int_T d2G/dn_x dn_y dA at x (centroid of the flat triangle T)."""
    reg = 0.0 + 0.0j
    for p, r in ((a, b), (b, c), (c, a)):
        pts, w = duffy_points(x, p, r, q)
        R = np.linalg.norm(pts - x, axis=-1)
        g = (np.exp(1j * k * R) * (1.0 - 1j * k * R) - 1.0) / R ** 3
        reg += (g * w).sum()
    return (fp_inv_r3(a, b, c, x) + reg) / FOUR_PI


def block(geom, k, alpha, target_shift, source_shift, self_block: bool, chunk: int = 1 << 15, rows=None):
    """Matrix block for collocation points of one cell (shifted by ``target_shift``)
    against the elements of one cell (shifted by ``source_shift``).  ``self_block``
    marks the block of a cell with itself (diagonal = self terms).  ``rows``
    restricts the targets to a subset of the cell's collocation points."""
    rows = np.arange(geom["centroid"].shape[0]) if rows is None else np.asarray(rows)
    x = geom["centroid"][rows] + np.asarray(target_shift)
    nx = geom["normal"][rows]
    sa = geom["a"] + np.asarray(source_shift)
    sb = geom["b"] + np.asarray(source_shift)
    sc = geom["c"] + np.asarray(source_shift)
    ny = geom["normal"]
    scen = geom["centroid"] + np.asarray(source_shift)
    n = scen.shape[0]
    dist = np.linalg.norm(x[:, None, :] - scen[None, :, :], axis=-1)
    order = rule_order(dist, geom["longest"][None, :])
    out = np.zeros((rows.size, n), dtype=np.complex128)
    if self_block:
        order[np.arange(rows.size), rows] = 0
    for q in (4, 8, 16):
        ia, jb = np.nonzero(order == q)
        for s in range(0, ia.size, chunk):
            i_ = ia[s:s + chunk]
            j_ = jb[s:s + chunk]
            pts, w = duffy_points(sa[j_], sb[j_], sc[j_], q)
            vals = kernels.bm_kernel(x[i_][:, None, :], pts, nx[i_][:, None, :], ny[j_][:, None, :], k, alpha)
            out[i_, j_] = (vals * w).sum(-1)
    if self_block:
        for r, i in enumerate(rows):
            hs = hypersingular_self(sa[i], sb[i], sc[i], x[r], k) if alpha != 0 else 0.0
            out[r, i] = 0.5 + alpha * hs
    return out


def near_offsets(grid, near_radius=(1, 1, 1)):
    """Near-field cell offsets d (target cell minus source cell): Chebyshev radius
    ``near_radius`` per axis, axes with a single cell dropped.  With radius 1 this
    gives the 3/9/27 unique near blocks of Sec. 3.2-3.3."""
    ranges = []
    for a in range(3):
        r = near_radius[a] if grid[a] > 1 else 0
        r = min(r, grid[a] - 1)
        ranges.append(range(-r, r + 1))
    return [(d1, d2, d3) for d3 in ranges[2] for d2 in ranges[1] for d1 in ranges[0]]


def near_blocks(vertices, triangles, lattice, k, alpha, near_radius=(1, 1, 1)):
    """S_d for every near offset d, computed once in cell-local coordinates with
    the source cell shifted by -d*pitch (translation invariance, Sec. 2.2/3.2)."""
    geom = element_geometry(vertices, triangles)
    pitch = np.asarray(lattice.pitch)
    out = {}
    for d in near_offsets(lattice.grid, near_radius):
        out[d] = block(geom, k, alpha, np.zeros(3), -np.asarray(d) * pitch, d == (0, 0, 0))
    return out


def dense_exact(vertices, triangles, lattice, k, alpha):
    """O1: the dense collocation matrix (eq. (matrixBEM) with Y = 0), every block
    integrated from absolute coordinates, no Toeplitz structure assumed."""
    geom = element_geometry(vertices, triangles)
    n = geom["centroid"].shape[0]
    C = lattice.n_cells
    A = np.zeros((C * n, C * n), dtype=np.complex128)
    for i in range(C):
        oi = lattice.cell_origin(i)
        for j in range(C):
            oj = lattice.cell_origin(j)
            A[i * n:(i + 1) * n, j * n:(j + 1) * n] = block(geom, k, alpha, oi, oj, i == j)
    return A


def collocation_points(vertices, triangles, lattice):
    """Absolute centroids and normals of all DOFs, ordered [cell][element]."""
    geom = element_geometry(vertices, triangles)
    C = lattice.n_cells
    pts = np.concatenate([geom["centroid"] + lattice.cell_origin(c) for c in range(C)])
    nrm = np.tile(geom["normal"], (C, 1))
    return pts, nrm


def rhs_plane_wave(vertices, triangles, lattice, k, alpha, directions, amplitude=1.0):
    """b = p_inc + alpha dp_inc/dn for p_inc = A e^{ik d.x} (eq. (planewave)); [R, N]."""
    x, n = collocation_points(vertices, triangles, lattice)
    out = []
    for d in np.atleast_2d(directions):
        p = amplitude * np.exp(1j * k * (x @ d))
        dp = 1j * k * (n @ d) * p
        out.append(p + alpha * dp)
    return np.array(out)


def rhs_point_source(vertices, triangles, lattice, k, alpha, sources, amplitude=1.0):
    """b for a monopole p_inc = A e^{ikR}/R, R = |x - s| (Sec. 4.2); [R, N]."""
    x, n = collocation_points(vertices, triangles, lattice)
    out = []
    for s in np.atleast_2d(sources):
        r = x - s
        R = np.linalg.norm(r, axis=1)
        p = amplitude * np.exp(1j * k * R) / R
        dp = amplitude * np.exp(1j * k * R) * (1j * k * R - 1.0) / R ** 2 * (r * n).sum(1) / R
        out.append(p + alpha * dp)
    return np.array(out)


# ---------------------------------------------------------------------------
# Post-processing: pressure at points in the fluid and insertion loss
# ---------------------------------------------------------------------------

def incident_plane_wave_at(points, k, directions, amplitude=1.0):
    """p_inc = A e^{ik d.x} (eq. (planewave)) at arbitrary points; [R, M]."""
    x = np.asarray(points, dtype=np.float64)
    return np.array([amplitude * np.exp(1j * k * (x @ np.asarray(d))) for d in np.atleast_2d(directions)])


def incident_point_source_at(points, k, sources, amplitude=1.0):
    """Monopole p_inc = A e^{ikR}/R, R = |x - s| (Sec. 4.2) at arbitrary points; [R, M]."""
    x = np.asarray(points, dtype=np.float64)
    out = []
    for s in np.atleast_2d(sources):
        R = np.linalg.norm(x - s, axis=1)
        out.append(amplitude * np.exp(1j * k * R) / R)
    return np.array(out)


def field_weights(vertices, triangles, lattice, k, points, chunk: int = 1 << 15):
    """W[m, j] = int_{Delta_j} dG/dn_y(x_m, y) dA(y) for every element j of every cell
    (ordered [cell][element], as the surface unknowns), the non-self Duffy rule of the
    module docstring chosen by |x_m - centroid_j| against the longest edge of j."""
    geom = element_geometry(vertices, triangles)
    x = np.asarray(points, dtype=np.float64)
    n = geom["centroid"].shape[0]
    C = lattice.n_cells
    W = np.zeros((x.shape[0], C * n), dtype=np.complex128)
    for c in range(C):
        o = lattice.cell_origin(c)
        sa, sb, sc = geom["a"] + o, geom["b"] + o, geom["c"] + o
        dist = np.linalg.norm(x[:, None, :] - (geom["centroid"] + o)[None, :, :], axis=-1)
        order = rule_order(dist, geom["longest"][None, :])
        for q in (4, 8, 16):
            im, jb = np.nonzero(order == q)
            for s in range(0, im.size, chunk):
                i_ = im[s:s + chunk]
                j_ = jb[s:s + chunk]
                pts, w = duffy_points(sa[j_], sb[j_], sc[j_], q)
                vals = kernels.dgreen_dny(x[i_][:, None, :], pts, geom["normal"][j_][:, None, :], k)
                W[i_, c * n + j_] = (vals * w).sum(-1)
    return W


def field(vertices, triangles, lattice, k, points, p_surface, p_inc=None):
    """Pressure at points x_m of the fluid from the surface pressure of a rigid scatterer:
    the CBIE (eq. (cbie)) with c(x) = 1 for x in the domain and dp/dn = 0 on the surface,

        p(x_m) = p_inc(x_m) - sum_j p_j int_{Delta_j} dG/dn_y(x_m, y) dA(y).

    p_surface: [R, N] (or [N]); p_inc: [R, M] at the points, or None for the scattered
    part alone.  Returns [R, M] (or [M])."""
    ps = np.asarray(p_surface, dtype=np.complex128)
    single = ps.ndim == 1
    ps = np.atleast_2d(ps)
    W = field_weights(vertices, triangles, lattice, k, points)
    out = -(ps @ W.T)
    if p_inc is not None:
        out = out + np.atleast_2d(p_inc)
    return out[0] if single else out


def insertion_loss(p_inc, p):
    """IL = 20 log10( sum_i |p_inc(x_i)| / sum_i |p(x_i)| ) over the observation points
    (eq. (insertionloss)); inputs [R, M] (or [M]), returns [R] (or a scalar)."""
    a = np.abs(np.asarray(p_inc)).sum(-1)
    b = np.abs(np.asarray(p)).sum(-1)
    return 20.0 * np.log10(a / b)
