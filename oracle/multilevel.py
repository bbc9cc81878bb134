"""FMPBEM2 (Sec. 3.3): the unique near blocks S_d of the FMPBEM approximated by a
multilevel FMM inside the unit cells (oracle; test infrastructure).

Reading of the subdivision (Sec. 3.3 with eq. (admissibility)): the box of a unit
cell is its lattice box (edge = pitch per axis, centred on the cell centre, which is
the origin of the cell mesh), halved along every axis ``levels`` times (uniform
depth: every leaf sits on level ``levels``).  An element belongs to the box holding
its centroid (its collocation point).  Boxes of one level of the whole lattice lie on
one regular grid, and two of them are well separated when their integer grid offset
has Chebyshev norm >= 2 (for cubic boxes that is |x_c - y_c| >= 2r with r the box
edge; the cells themselves, level 0, are near exactly when that norm is <= 1, the
near set of Sec. 3.2).

Approximated block, by its plain definition: for target cell i, source cell i - d
and leaves a (target) and b (source), take the coarsest level l whose ancestors of a
and b are well separated.  None: the exact entries of S_d (P2P).  Otherwise

    S~_d[a, b] = U_a  L2L(level l -> leaves along a)  K(x_c - y_c)  M2M(leaves -> level l along b)  V_b

with V_b the P2M of eq. (p2m) about the centre of leaf b, U_a the L2P of eq. (l2p)
about the centre of leaf a, M2M / L2L of eqs. (m2m) / (l2l) between the centres of
consecutive ancestors and K the M2L of eq. (m2l) between the two level-l boxes
(centre offset including the lattice offset d * pitch).  The truncation number is
n_t,near, independent of the n_t of the cell-level far field (Sec. 3.3).
The far field of the cells (offsets outside the near set) is the FMPBEM's.
"""
from __future__ import annotations

import numpy as np

from . import bem, fmm
from .operator import FMPBEM, sampled_apply, grid_coords


class CellTree:
    """Uniform-depth subdivision of the lattice box of a unit cell."""

    def __init__(self, vertices, triangles, pitch, levels: int):
        geom = bem.element_geometry(vertices, triangles)
        self.pitch = np.asarray(pitch, dtype=np.float64)
        self.levels = int(levels)
        cen = geom["centroid"]
        if np.any(np.abs(cen) > 0.5 * self.pitch[None, :]):
            raise ValueError("a collocation point lies outside the cell's lattice box")
        nl = 1 << self.levels
        leaf = np.floor((cen + 0.5 * self.pitch) / (self.pitch / nl)).astype(np.int64)
        self.leaf = np.clip(leaf, 0, nl - 1)          # [n, 3] leaf grid coordinates

    def coords(self, level: int):
        """[n, 3] grid coordinates of every element's box on ``level``."""
        return self.leaf >> (self.levels - level)

    def centre(self, level: int, c):
        """Centre of the box with grid coordinates c on ``level`` (cell-local)."""
        h = self.pitch / (1 << level)
        return -0.5 * self.pitch + (np.asarray(c, dtype=np.float64) + 0.5) * h

    def leaves(self):
        """{leaf grid coordinates (tuple): element indices}."""
        out = {}
        for e, c in enumerate(map(tuple, self.leaf)):
            out.setdefault(c, []).append(e)
        return {c: np.array(v) for c, v in out.items()}


def interaction_level(tree: CellTree, ca, cb, d):
    """Coarsest level whose ancestors of leaves ca (target) and cb (source) are well
    separated for cell offset d, or None (near on every level: P2P)."""
    for lev in range(tree.levels + 1):
        sh = tree.levels - lev
        delta = (np.asarray(ca) >> sh) - (np.asarray(cb) >> sh) + np.asarray(d) * (1 << lev)
        if np.max(np.abs(delta)) >= 2:
            return lev
    return None


def approx_blocks(vertices, triangles, lattice, k, alpha, levels, near_order, near_radius=(1, 1, 1), exact=None):
    """S~_d (dense, n x n) for every near offset d, composed leaf pair by leaf pair.
    ``exact``: the exact blocks S_d when already computed."""
    if tuple(near_radius) != (1, 1, 1):
        raise ValueError("the multilevel near field takes near radius 1")
    tree = CellTree(vertices, triangles, lattice.pitch, levels)
    pitch = tree.pitch
    S = exact if exact is not None else bem.near_blocks(vertices, triangles, lattice, k, alpha, near_radius)
    t = np.asarray(triangles)
    leaves = tree.leaves()
    L = tree.levels
    V = {c: fmm.p2m(vertices, t[e], k, near_order, center=tree.centre(L, c)) for c, e in leaves.items()}
    U = {c: fmm.l2p(vertices, t[e], k, near_order, alpha, center=tree.centre(L, c)) for c, e in leaves.items()}

    # translation matrices by shift vector, and the chains per (leaf, level), formed once
    cache = {}

    def translation(kind, vec):
        key = (kind,) + tuple(np.round(np.asarray(vec) / pitch * (1 << (L + 2))).astype(int))
        if key not in cache:
            fn = {"m2m": fmm.m2m, "l2l": fmm.l2l, "m2l": fmm.m2l}[kind]
            cache[key] = fn(vec, k, near_order)[0]
        return cache[key]

    def up(c, lev):
        """M2M chain: moments of leaf c's box re-centred on its ancestor of level ``lev``."""
        key = ("up", c, lev)
        if key not in cache:
            T = np.eye(fmm.n_coeffs(near_order), dtype=np.complex128)
            cc = np.asarray(c)
            for l in range(L, lev, -1):
                T = translation("m2m", tree.centre(l, cc) - tree.centre(l - 1, cc >> 1)) @ T
                cc = cc >> 1
            cache[key] = T @ V[c]
        return cache[key]

    def down(c, lev):
        """L2L chain: local coefficients of the level-``lev`` ancestor of leaf c moved to c."""
        key = ("down", c, lev)
        if key not in cache:
            T = np.eye(fmm.n_coeffs(near_order), dtype=np.complex128)
            path = [np.asarray(c) >> (L - l) for l in range(lev, L + 1)]
            for l in range(lev, L):
                T = translation("l2l", tree.centre(l + 1, path[l - lev + 1]) - tree.centre(l, path[l - lev])) @ T
            cache[key] = U[c] @ T
        return cache[key]

    out = {}
    for d, Sd in S.items():
        A = np.zeros_like(Sd)
        for ca, ea in leaves.items():
            for cb, eb in leaves.items():
                lev = interaction_level(tree, ca, cb, d)
                if lev is None:
                    A[np.ix_(ea, eb)] = Sd[np.ix_(ea, eb)]
                    continue
                sh = L - lev
                D = tree.centre(lev, np.asarray(ca) >> sh) - tree.centre(lev, np.asarray(cb) >> sh) + np.asarray(d) * pitch
                A[np.ix_(ea, eb)] = down(ca, lev) @ translation("m2l", D) @ up(cb, lev)
        out[d] = A
    return out


class FMPBEM2(FMPBEM):
    """The FMPBEM with every near block replaced by its multilevel approximation."""

    def __init__(self, vertices, triangles, lattice, k, order, alpha, levels, near_order, near_radius=(1, 1, 1)):
        super().__init__(vertices, triangles, lattice, k, order, alpha, near_radius)
        self.levels = levels
        self.near_order = near_order
        self.S_exact = self.S
        self.S = approx_blocks(vertices, triangles, lattice, k, alpha, levels, near_order, near_radius,
                               exact=self.S_exact)


def sampled_apply2(vertices, triangles, lattice, k, order, alpha, levels, near_order, x, dofs):
    """(A2 x)[:, dof] of the FMPBEM2 operator for the listed DOFs only, for lattices whose
    near blocks are too large to form: the far field as in operator.sampled_apply, the near
    field leaf pair by leaf pair as in approx_blocks (exact row entries for P2P pairs,
    U_a L2L K M2M V_b otherwise), restricted to the listed rows.  x: [R, C, n]."""
    x = np.asarray(x, dtype=np.complex128)
    grid = tuple(lattice.grid)
    n = int(np.asarray(triangles).shape[0])
    R = x.shape[0]
    tree = CellTree(vertices, triangles, lattice.pitch, levels)
    pitch = tree.pitch
    L = tree.levels
    t = np.asarray(triangles)
    geom = bem.element_geometry(vertices, triangles)
    leaves = tree.leaves()
    leaf_of = {int(e): c for c, es in leaves.items() for e in es}
    # P2M of every element about its leaf centre (one batched evaluation)
    Vall = fmm.p2m(vertices, t, k, near_order, center=tree.centre(L, tree.leaf))
    V = {c: Vall[:, e] for c, e in leaves.items()}
    g = grid_coords(grid)
    gsz = np.asarray(grid)
    dofs = [int(v) for v in dofs]
    out = sampled_apply(vertices, triangles, lattice, k, order, alpha, x, dofs, with_near=False)
    cache = {}

    def translation(kind, vec):
        key = (kind,) + tuple(np.round(np.asarray(vec) / pitch * (1 << (L + 2))).astype(int))
        if key not in cache:
            fn = {"m2m": fmm.m2m, "l2l": fmm.l2l, "m2l": fmm.m2l}[kind]
            cache[key] = fn(vec, k, near_order)[0]
        return cache[key]

    def up(c, lev):
        key = ("up", c, lev)
        if key not in cache:
            T = np.eye(fmm.n_coeffs(near_order), dtype=np.complex128)
            cc = np.asarray(c)
            for l in range(L, lev, -1):
                T = translation("m2m", tree.centre(l, cc) - tree.centre(l - 1, cc >> 1)) @ T
                cc = cc >> 1
            cache[key] = T @ V[c]
        return cache[key]

    def down_row(a, c, lev):
        """Row of U_a L2L(level lev -> leaf c) for element a of leaf c."""
        if ("u", a) not in cache:
            cache[("u", a)] = fmm.l2p(vertices, t[[a]], k, near_order, alpha, center=tree.centre(L, c))[0]
        u = cache[("u", a)]
        path = [np.asarray(c) >> (L - l) for l in range(lev, L + 1)]
        T = np.eye(fmm.n_coeffs(near_order), dtype=np.complex128)
        for l in range(lev, L):
            T = translation("l2l", tree.centre(l + 1, path[l - lev + 1]) - tree.centre(l, path[l - lev])) @ T
        return u @ T

    near = bem.near_offsets(grid)
    for s, dof in enumerate(dofs):
        i, a = divmod(dof, n)
        ca = leaf_of[a]
        acc = np.zeros(R, dtype=np.complex128)
        for d in near:
            src = g[i] - np.asarray(d)
            if not np.all((src >= 0) & (src < gsz)):
                continue
            j = int(src[0] + grid[0] * (src[1] + grid[1] * src[2]))
            xs = x[:, j, :]
            exact = None
            rows = {}
            for cb, eb in leaves.items():
                lev = interaction_level(tree, ca, cb, d)
                if lev is None:
                    if exact is None:
                        exact = bem.block(geom, k, alpha, np.zeros(3), -np.asarray(d) * pitch, d == (0, 0, 0),
                                          rows=[a])[0]
                    acc += xs[:, eb] @ exact[eb]
                    continue
                sh = L - lev
                D = tree.centre(lev, np.asarray(ca) >> sh) - tree.centre(lev, np.asarray(cb) >> sh) + np.asarray(d) * pitch
                key = (lev,) + tuple(np.round(D / pitch * (1 << (L + 2))).astype(int))
                if key not in rows:
                    rows[key] = down_row(a, ca, lev) @ translation("m2l", D)
                acc += (xs[:, eb] @ up(cb, lev).T) @ rows[key]
        out[:, s] += acc
    return out
