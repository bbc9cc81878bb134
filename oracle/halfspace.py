"""Half-space variant of the BEM and of the FMPBEM operator (oracle; test infrastructure).

Green's function of the half-space (Sec. 2.1, eq. (green3dHalf)):
    G_h(x, y) = G(x, y) + R_p G(x, y^),   y^ = mirror image of y in the plane z = z_g,
with R_p the reflection coefficient.  The collocation matrix splits into the
full-space part and an image part (Sec. 2.3, eq. (toeplitzBEMsymmetry)); in the
image part the source element is the mirrored element, whose outward normal is
the mirrored normal, so d/dn_y G(x, y^) is the normal derivative at the image
point along the mirrored normal (and alpha d2/dn_x dn_y likewise for eq. (bm)).

Readings (Sec. 3.4).  The plane is z = z_g, normal to the third lattice axis.
  * First case, the plane parallel to every periodic direction (grid[2] == 1): the image part is
    block Toeplitz like the direct part; the block of target cell i and source cell j depends
    on d = i - j through the image offset t^_d = (d1 p1, d2 p2, -2 z_g).
  * Second case, periodicity along z (grid[2] > 1): the image of source cell j sits at
    z = 2 z_g - j3 p3, so the block depends on (d1, d2, s = i3 + j3) (block Hankel along z),
    t^ = (d1 p1, d2 p2, s p3 - 2 z_g).  Reversing the source cells along z (P x, cell index
    M3 - 1 - j3) turns it into a Toeplitz product in e = i3 - (M3 - 1 - j3) = s - (M3 - 1), the
    column permutation of Sec. 2.3 and Sec. 3.5.
Near / far for the image part (eq. (admissibilityMirror)), in the Chebyshev reading of the
direct part: an image block is near when |d1| <= r1, |d2| <= r2 and its z offset
|s p3 - 2 z_g| < (r3 + 1) p3 (r = near radius, p = pitch; s = 0 in the first case);
otherwise it is applied through the multipole chain.  The multipole moments of a mirrored
cell about its mirrored centre are D_z V0 x with D_z = diag((-1)^(n+m)) (a reflection in z
maps theta to pi - theta, and Y_n^m to (-1)^(n+m) Y_n^m), so the far image block is
U0 K(t^) D_z V0 (Appendix A, eq. (greenFMMhalfspace); U and V are shared by both parts).
The surface of the whole lattice must not cross the plane.

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
    lo = z.min()
    hi = z.max() + (lattice.grid[2] - 1) * lattice.pitch[2]
    if not (lo >= zg or hi <= zg):
        raise ValueError("the surface crosses the plane")


def all_offsets(grid):
    """Image offsets (d1, d2, s): d = target - source in x, y; s = target + source along z."""
    return [(d1, d2, s) for s in range(0, 2 * grid[2] - 1) for d2 in range(-(grid[1] - 1), grid[1])
            for d1 in range(-(grid[0] - 1), grid[0])]


def image_near_offsets(grid, pitch, zg, near_radius=(1, 1, 1)):
    r1 = min(near_radius[0], grid[0] - 1)
    r2 = min(near_radius[1], grid[1] - 1)
    return [o for o in all_offsets(grid)
            if abs(o[0]) <= r1 and abs(o[1]) <= r2 and abs(o[2] * pitch[2] - 2.0 * zg) < (near_radius[2] + 1) * pitch[2]]


def image_offset_vector(o, pitch, zg):
    return np.array([o[0] * pitch[0], o[1] * pitch[1], o[2] * pitch[2] - 2.0 * zg])


def image_blocks(vertices, triangles, lattice, k, alpha, zg, offsets):
    """Image blocks for the listed offsets (d1, d2, s), in the target cell's local coordinates:
    the source cell shifted by (-d1 p1, -d2 p2) and by s p3 along z relative to the target's
    lattice position (source z + target z = s p3), then mirrored in the plane z = z_g."""
    geom = bem.element_geometry(vertices, triangles)
    pitch = np.asarray(lattice.pitch)
    out = {}
    for o in offsets:
        shift = np.array([-o[0] * pitch[0], -o[1] * pitch[1], o[2] * pitch[2]])
        mgeom = mirrored_geometry(np.asarray(vertices) + shift, triangles, zg)
        out[o] = cross_block(geom, mgeom, k, alpha, np.zeros(3), np.zeros(3))
    return out


def image_pairs(grid, o):
    """(target cells, source cells) with target - source = (d1, d2) and target + source = s."""
    g = grid_coords(grid)
    src = np.stack([g[:, 0] - o[0], g[:, 1] - o[1], o[2] - g[:, 2]], 1)
    ok = np.all((src >= 0) & (src < np.asarray(grid)[None, :]), axis=1)
    tgt = np.nonzero(ok)[0]
    s = src[ok]
    return tgt, s[:, 0] + grid[0] * (s[:, 1] + grid[1] * s[:, 2])


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
            # the mirror of cell j's elements
            mgeom = mirrored_geometry(np.asarray(vertices) + oj, triangles, zg)
            A[i * n:(i + 1) * n, j * n:(j + 1) * n] += rp * cross_block(geom, mgeom, k, alpha, oi, np.zeros(3))
    return A


class FMPBEMHalfSpace(FMPBEM):
    """The FMPBEM operator of eq. (2dPeriodicFMM_halfspace): (S + U K V) + R_p (S^ + U K^ D_z V),
    the image blocks keyed by (d1, d2, s) (both cases of Sec. 3.4)."""

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
            t = np.array([image_offset_vector(o, pitch, zg) for o in self.img_far])
            Ks = fmm.m2l(t, k, order) * D[None, None, :]
        else:
            Ks = np.zeros((0, self.p, self.p), dtype=np.complex128)
        self.Kimg = {o: Ks[i] for i, o in enumerate(self.img_far)}
        self._ipairs = {o: image_pairs(self.grid, o) for o in self.img_near + self.img_far}

    def image_key(self, i, j):
        g = grid_coords(self.grid)
        return (int(g[i][0] - g[j][0]), int(g[i][1] - g[j][1]), int(g[i][2] + g[j][2]))

    def near_apply(self, x):
        y = super().near_apply(x)
        for o in self.img_near:
            t, s = self._ipairs[o]
            y[:, t, :] += self.rp * (x[:, s, :] @ self.Simg[o].T)
        return y

    def far_apply(self, x):
        y = super().far_apply(x)
        m = x @ self.V0.T
        loc = np.zeros(m.shape, dtype=np.complex128)
        for o in self.img_far:
            t, s = self._ipairs[o]
            loc[:, t, :] += m[:, s, :] @ self.Kimg[o].T
        return y + self.rp * (loc @ self.U0.T)

    def dense(self):
        A = super().dense()
        C, n = self.n_cells, self.n
        for i in range(C):
            for j in range(C):
                o = self.image_key(i, j)
                blk = self.Simg[o] if o in self.Simg else self.U0 @ self.Kimg[o] @ self.V0
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
    # mirrored lattice surface: each cell's shifted vertices mirrored, order (a, c, b)
    from workloads import Lattice
    one = Lattice((1, 1, 1), lattice.pitch)
    tm = np.asarray(triangles)[:, [0, 2, 1]]
    Wm = np.concatenate([bem.field_weights(mirror_points(np.asarray(vertices) + lattice.cell_origin(c), zg), tm,
                                           one, k, points) for c in range(lattice.n_cells)], axis=1)
    out = -(ps @ (W + rp * Wm).T)
    if p_inc is not None:
        out = out + np.atleast_2d(p_inc)
    return out
