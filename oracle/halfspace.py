"""Half-space variant of the BEM and of the FMPBEM operator (oracle; test infrastructure).

Green's function of the half-space (Sec. 2.1, eq. (green3dHalf)):
    G_h(x, y) = G(x, y) + R_p G(x, y^),   y^ = mirror image of y in the plane z = z_g,
with R_p the reflection coefficient.  The collocation matrix splits into the
full-space part and an image part (Sec. 2.3, eq. (toeplitzBEMsymmetry)); in the
image part the source element is the mirrored element, whose outward normal is
the mirrored normal, so d/dn_y G(x, y^) is the normal derivative at the image
point along the mirrored normal (and alpha d2/dn_x dn_y likewise for eq. (bm)).

Reading (Sec. 3.4, first case): the plane is parallel to every periodic direction,
i.e. the lattice has one layer of cells along z (grid[2] == 1) and the plane is
z = z_g.  The image part is then block Toeplitz like the direct part: the image
of source cell j sits at the mirrored centre, and the block of target cell i and
source cell j depends on d = i - j only, through the image offset
    t^_d = (d1 p1, d2 p2, -2 z_g).
Near / far for the image part (eq. (admissibilityMirror)), in the same Chebyshev
reading as the direct part: the image block is near when |d1| <= r1, |d2| <= r2
and |2 z_g| < (r3 + 1) p3 (r = near radius, p = pitch); otherwise it is applied
through the multipole chain.  The multipole moments of a mirrored cell about its
mirrored centre are D_z V0 x with D_z = diag((-1)^(n+m)) (a reflection in z maps
theta to pi - theta, and Y_n^m to (-1)^(n+m) Y_n^m), so the far image block is
U0 K(t^_d) D_z V0 (Appendix A, eq. (greenFMMhalfspace); U and V are shared by
both parts).  The surface must not cross the plane.

Incident fields in the half-space are the free field plus R_p times its mirror
image: a point source s gets the image source s^, a plane wave A e^{ik d.x} gets
R_p A e^{ik d.(Mx)} = R_p A e^{2ik z_g d3} e^{ik (Md).x}, M = diag(1, 1, -1).
"""
from __future__ import annotations

import numpy as np

from . import bem, fmm, kernels
from .operator import FMPBEM, grid_coords, pairs
from .quadrature import duffy_points


def mirror_points(v, zg):
    out = np.array(v, dtype=np.float64, copy=True)
    out[..., 2] = 2.0 * zg - out[..., 2]
    return out


def mirrored_geometry(vertices, triangles, zg):
    """Element geometry of the mirrored surface, vertices (a, c, b) so that the
    normal is the mirror of the original normal (a reflection reverses the
    orientation of (a, b, c)); the Duffy rule collapsed at a is the same point set."""
    t = np.asarray(triangles)
    return bem.element_geometry(mirror_points(vertices, zg), t[:, [0, 2, 1]])


def dz_signs(order):
    """(-1)^(n+m) for all (n, m), index n^2 + n + m."""
    out = []
    for n in range(order + 1):
        for m in range(-n, n + 1):
            out.append(-1.0 if (n + m) % 2 else 1.0)
    return np.array(out)


def cross_block(tgeom, sgeom, k, alpha, target_shift, source_shift, chunk: int = 1 << 15, rows=None):
    """int_{Delta_j} [dG/dn_y + alpha d2G/dn_x dn_y](x_i, y) dA(y) for collocation points of
    ``tgeom`` (shifted) against the elements of ``sgeom`` (shifted), with the non-self Duffy
    rule of bem (no element of one surface coincides with one of the other)."""
    rows = np.arange(tgeom["centroid"].shape[0]) if rows is None else np.asarray(rows)
    x = tgeom["centroid"][rows] + np.asarray(target_shift)
    nx = tgeom["normal"][rows]
    sa = sgeom["a"] + np.asarray(source_shift)
    sb = sgeom["b"] + np.asarray(source_shift)
    sc = sgeom["c"] + np.asarray(source_shift)
    ny = sgeom["normal"]
    scen = sgeom["centroid"] + np.asarray(source_shift)
    dist = np.linalg.norm(x[:, None, :] - scen[None, :, :], axis=-1)
    order = bem.rule_order(dist, sgeom["longest"][None, :])
    out = np.zeros((rows.size, scen.shape[0]), dtype=np.complex128)
    for q in (4, 8, 16):
        ia, jb = np.nonzero(order == q)
        for s in range(0, ia.size, chunk):
            i_ = ia[s:s + chunk]
            j_ = jb[s:s + chunk]
            pts, w = duffy_points(sa[j_], sb[j_], sc[j_], q)
            vals = kernels.bm_kernel(x[i_][:, None, :], pts, nx[i_][:, None, :], ny[j_][:, None, :], k, alpha)
            out[i_, j_] = (vals * w).sum(-1)
    return out


def check_side(vertices, lattice, zg):
    z = np.asarray(vertices)[:, 2]
    if lattice.grid[2] != 1:
        raise ValueError("the plane must be parallel to every periodic direction (grid[2] == 1)")
    if not (np.all(z >= zg) or np.all(z <= zg)):
        raise ValueError("the surface crosses the plane")


def image_near_offsets(grid, pitch, zg, near_radius=(1, 1, 1)):
    if abs(2.0 * zg) >= (near_radius[2] + 1) * pitch[2]:
        return []
    r1 = min(near_radius[0], grid[0] - 1)
    r2 = min(near_radius[1], grid[1] - 1)
    return [(d1, d2, 0) for d2 in range(-r2, r2 + 1) for d1 in range(-r1, r1 + 1)]


def all_offsets(grid):
    return [(d1, d2, 0) for d2 in range(-(grid[1] - 1), grid[1]) for d1 in range(-(grid[0] - 1), grid[0])]


def image_blocks(vertices, triangles, lattice, k, alpha, zg, offsets):
    """Image blocks for the listed offsets d (target cell minus source cell), in cell-local
    coordinates: target at the origin, mirrored source cell shifted by -d*pitch in x, y."""
    geom = bem.element_geometry(vertices, triangles)
    mgeom = mirrored_geometry(vertices, triangles, zg)
    pitch = np.asarray(lattice.pitch)
    return {d: cross_block(geom, mgeom, k, alpha, np.zeros(3), -np.asarray(d) * pitch) for d in offsets}


def dense_exact(vertices, triangles, lattice, k, alpha, zg, rp):
    """O1 in the half-space: every block of G_h integrated from absolute coordinates."""
    check_side(vertices, lattice, zg)
    A = bem.dense_exact(vertices, triangles, lattice, k, alpha)
    geom = bem.element_geometry(vertices, triangles)
    n = geom["centroid"].shape[0]
    C = lattice.n_cells
    for i in range(C):
        oi = lattice.cell_origin(i)
        for j in range(C):
            oj = lattice.cell_origin(j)
            # the mirror of cell j's elements: mirror the shifted vertices (z shifts are zero)
            mgeom = mirrored_geometry(np.asarray(vertices) + oj, triangles, zg)
            A[i * n:(i + 1) * n, j * n:(j + 1) * n] += rp * cross_block(geom, mgeom, k, alpha, oi, np.zeros(3))
    return A


class FMPBEMHalfSpace(FMPBEM):
    """The FMPBEM operator of eq. (2dPeriodicFMM_halfspace) for the first case of Sec. 3.4:
    (S + U K V) + R_p (S^ + U K^ D_z V), blocks by offset d."""

    def __init__(self, vertices, triangles, lattice, k, order, alpha, zg, rp, near_radius=(1, 1, 1)):
        check_side(vertices, lattice, zg)
        super().__init__(vertices, triangles, lattice, k, order, alpha, near_radius)
        self.zg = float(zg)
        self.rp = complex(rp)
        pitch = np.asarray(lattice.pitch, dtype=np.float64)
        self.img_near = image_near_offsets(self.grid, pitch, zg, near_radius)
        self.Simg = image_blocks(vertices, triangles, lattice, k, alpha, zg, self.img_near)
        self.img_far = [d for d in all_offsets(self.grid) if d not in set(self.img_near)]
        D = dz_signs(order)
        if self.img_far:
            t = np.asarray(self.img_far, dtype=np.float64) * pitch[None, :]
            t[:, 2] = -2.0 * zg
            Ks = fmm.m2l(t, k, order) * D[None, None, :]
        else:
            Ks = np.zeros((0, self.p, self.p), dtype=np.complex128)
        self.Kimg = {d: Ks[i] for i, d in enumerate(self.img_far)}
        for d in self.img_near + self.img_far:
            if d not in self._pairs:
                self._pairs[d] = pairs(self.grid, d)

    def near_apply(self, x):
        y = super().near_apply(x)
        for d in self.img_near:
            t, s = self._pairs[d]
            y[:, t, :] += self.rp * (x[:, s, :] @ self.Simg[d].T)
        return y

    def far_apply(self, x):
        y = super().far_apply(x)
        m = x @ self.V0.T
        loc = np.zeros(m.shape, dtype=np.complex128)
        for d in self.img_far:
            t, s = self._pairs[d]
            loc[:, t, :] += m[:, s, :] @ self.Kimg[d].T
        return y + self.rp * (loc @ self.U0.T)

    def dense(self):
        A = super().dense()
        C, n = self.n_cells, self.n
        g = grid_coords(self.grid)
        for i in range(C):
            for j in range(C):
                d = tuple(int(v) for v in (g[i] - g[j]))
                blk = self.Simg[d] if d in self.Simg else self.U0 @ self.Kimg[d] @ self.V0
                A[i * n:(i + 1) * n, j * n:(j + 1) * n] += self.rp * blk
        return A


def rhs_plane_wave(vertices, triangles, lattice, k, alpha, directions, zg, rp, amplitude=1.0):
    """b for p_inc = A e^{ik d.x} plus its reflection R_p A e^{ik d.(Mx)}; [R, N]."""
    out = []
    for d in np.atleast_2d(directions):
        dm = np.array([d[0], d[1], -d[2]])
        a_img = rp * amplitude * np.exp(2j * k * zg * d[2])
        out.append(bem.rhs_plane_wave(vertices, triangles, lattice, k, alpha, [d], amplitude)[0] +
                   bem.rhs_plane_wave(vertices, triangles, lattice, k, alpha, [dm], a_img)[0])
    return np.array(out)


def rhs_point_source(vertices, triangles, lattice, k, alpha, sources, zg, rp, amplitude=1.0):
    """b for a monopole at s plus R_p times a monopole at the image source; [R, N]."""
    src = np.atleast_2d(sources)
    return (bem.rhs_point_source(vertices, triangles, lattice, k, alpha, src, amplitude) +
            bem.rhs_point_source(vertices, triangles, lattice, k, alpha, mirror_points(src, zg), rp * amplitude))


def incident_plane_wave_at(points, k, directions, zg, rp, amplitude=1.0):
    pts = np.asarray(points, dtype=np.float64)
    return (bem.incident_plane_wave_at(pts, k, directions, amplitude) +
            rp * bem.incident_plane_wave_at(mirror_points(pts, zg), k, directions, amplitude))


def incident_point_source_at(points, k, sources, zg, rp, amplitude=1.0):
    return (bem.incident_point_source_at(points, k, sources, amplitude) +
            rp * bem.incident_point_source_at(points, k, mirror_points(np.atleast_2d(sources), zg), amplitude))


def field(vertices, triangles, lattice, k, points, p_surface, zg, rp, p_inc=None):
    """p(x_m) = p_inc(x_m) - sum_j p_j [W_j(x_m) + R_p W^_j(x_m)], W^ over the mirrored elements
    (eq. (cbie) with c = 1 and the half-space Green's function)."""
    ps = np.atleast_2d(np.asarray(p_surface, dtype=np.complex128))
    W = bem.field_weights(vertices, triangles, lattice, k, points)
    # mirrored lattice surface: mirror each cell's shifted vertices (z shifts are zero), reversed order
    Wm = bem.field_weights(mirror_points(vertices, zg), np.asarray(triangles)[:, [0, 2, 1]], lattice, k, points)
    out = -(ps @ (W + rp * Wm).T)
    if p_inc is not None:
        out = out + np.atleast_2d(p_inc)
    return out
