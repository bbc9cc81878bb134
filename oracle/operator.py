"""O2: the FMPBEM operator S + U K V applied block by block, without any FFT
(oracle; test infrastructure).

Structure (Sec. 3.2, eq. (2dPeriodicFMM)): cells are the FMM boxes; for a
target cell i and a source cell j with offset d = i - j,
  * d in the near set (Chebyshev distance <= 1 per periodic axis, the
    admissibility reading of eq. (admissibility) that yields the 9 unique near
    blocks of Sec. 3.3):   block = S_d
  * otherwise:             block = U0 K_d V0
Cell index c = i1 + M1 (i2 + M2 i3); DOF index = c * n + element.
"""
from __future__ import annotations

import numpy as np

from . import bem, fmm


def grid_coords(grid):
    M1, M2, M3 = grid
    c = np.arange(M1 * M2 * M3)
    return np.stack([c % M1, (c // M1) % M2, c // (M1 * M2)], 1)


def far_offsets(grid, near):
    near = set(near)
    out = []
    for d3 in range(-(grid[2] - 1), grid[2]):
        for d2 in range(-(grid[1] - 1), grid[1]):
            for d1 in range(-(grid[0] - 1), grid[0]):
                if (d1, d2, d3) not in near:
                    out.append((d1, d2, d3))
    return out


def pairs(grid, d):
    """(target cells, source cells) with target - source = d, both inside the grid."""
    g = grid_coords(grid)
    src = g - np.asarray(d)[None, :]
    ok = np.all((src >= 0) & (src < np.asarray(grid)[None, :]), axis=1)
    tgt = np.nonzero(ok)[0]
    s = src[ok]
    return tgt, s[:, 0] + grid[0] * (s[:, 1] + grid[1] * s[:, 2])


class FMPBEM:
    """All blocks of the FMPBEM operator for one lattice / frequency / order."""

    def __init__(self, vertices, triangles, lattice, k, order, alpha, near_radius=(1, 1, 1)):
        self.lattice = lattice
        self.grid = tuple(lattice.grid)
        self.k = k
        self.order = order
        self.alpha = alpha
        self.n = int(np.asarray(triangles).shape[0])
        self.p = fmm.n_coeffs(order)
        self.near = bem.near_offsets(self.grid, near_radius)
        self.S = bem.near_blocks(vertices, triangles, lattice, k, alpha, near_radius)
        self.V0 = fmm.p2m(vertices, triangles, k, order)
        self.U0 = fmm.l2p(vertices, triangles, k, order, alpha)
        self.far = far_offsets(self.grid, self.near)
        pitch = np.asarray(lattice.pitch)
        if self.far:
            Ks = fmm.m2l(np.asarray(self.far, dtype=np.float64) * pitch[None, :], k, order)
        else:
            Ks = np.zeros((0, self.p, self.p), dtype=np.complex128)
        self.K = {d: Ks[i] for i, d in enumerate(self.far)}
        self._pairs = {d: pairs(self.grid, d) for d in self.near + self.far}

    @classmethod
    def from_workload(cls, w, alpha=None):
        if alpha is None:
            alpha = bem.default_alpha(w.k, w.formulation)
        return cls(w.vertices, w.triangles, w.lattice, w.k, w.order, alpha, w.near_radius)

    @property
    def n_cells(self):
        return self.lattice.n_cells

    def near_apply(self, x):
        """sum over near offsets of S_d x_{i-d}; x [R, C, n] -> [R, C, n]."""
        y = np.zeros_like(x)
        for d in self.near:
            t, s = self._pairs[d]
            y[:, t, :] += x[:, s, :] @ self.S[d].T
        return y

    def far_apply(self, x):
        """U0 sum over far offsets of K_d V0 x_{i-d}; x [R, C, n] -> [R, C, n]."""
        m = x @ self.V0.T
        loc = np.zeros(m.shape, dtype=np.complex128)
        for d in self.far:
            t, s = self._pairs[d]
            loc[:, t, :] += m[:, s, :] @ self.K[d].T
        return loc @ self.U0.T

    def matvec(self, x):
        """y = (S + U K V) x for x of shape [N], [R, N] or [R, C, n]."""
        x = np.asarray(x, dtype=np.complex128)
        shape = x.shape
        xr = x.reshape(-1, self.n_cells, self.n)
        y = self.near_apply(xr) + self.far_apply(xr)
        return y.reshape(shape)

    def dense(self):
        """All blocks materialised: [N, N] (small lattices only)."""
        C, n = self.n_cells, self.n
        A = np.zeros((C * n, C * n), dtype=np.complex128)
        g = grid_coords(self.grid)
        for i in range(C):
            for j in range(C):
                d = tuple(int(v) for v in (g[i] - g[j]))
                blk = self.S[d] if d in self.S else self.U0 @ self.K[d] @ self.V0
                A[i * n:(i + 1) * n, j * n:(j + 1) * n] = blk
        return A

    def row(self, dof: int):
        """One row of the operator, computed from the blocks: [N]."""
        C, n = self.n_cells, self.n
        i, a = divmod(dof, n)
        g = grid_coords(self.grid)
        out = np.zeros(C * n, dtype=np.complex128)
        ua = self.U0[a]
        for j in range(C):
            d = tuple(int(v) for v in (g[i] - g[j]))
            out[j * n:(j + 1) * n] = self.S[d][a] if d in self.S else (ua @ self.K[d]) @ self.V0
        return out


def sampled_apply(vertices, triangles, lattice, k, order, alpha, x, dofs, near_radius=(1, 1, 1), chunk=256,
                  with_near=True):
    """(A x)[:, dof] of the O2 operator for the listed DOFs only, for lattices too large
    to materialise S_d.  Near field: for every cell holding a listed DOF, the rows of its
    near blocks S_d at the listed elements, each integrated for its collocation point
    alone.  Far field: U0[a] sum_j K_{i-j} V0 x_j, the translations K_d formed ``chunk``
    offsets at a time so that memory stays bounded on large lattices.  ``with_near=False``:
    the far field alone.
    x: [R, C, n]; returns [R, len(dofs)]."""
    x = np.asarray(x, dtype=np.complex128)
    grid = tuple(lattice.grid)
    n = int(np.asarray(triangles).shape[0])
    R = x.shape[0]
    geom = bem.element_geometry(vertices, triangles)
    pitch = np.asarray(lattice.pitch)
    V0 = fmm.p2m(vertices, triangles, k, order)
    U0 = fmm.l2p(vertices, triangles, k, order, alpha)
    near = bem.near_offsets(grid, near_radius)
    far = far_offsets(grid, near)
    g = grid_coords(grid)
    gsz = np.asarray(grid)
    dofs = [int(v) for v in dofs]
    cells = sorted(set(d // n for d in dofs))

    def source(i, d):
        src = g[i] - np.asarray(d)
        if np.all((src >= 0) & (src < gsz)):
            return int(src[0] + grid[0] * (src[1] + grid[1] * src[2]))
        return None

    # near field: y_near[i][:, a] = sum_d S_d[a] x_{i-d}
    near_val = {}
    for i in cells:
        rows = sorted(set(d % n for d in dofs if d // n == i))
        acc = np.zeros((R, len(rows)), dtype=np.complex128)
        for d in (near if with_near else []):
            j = source(i, d)
            if j is None:
                continue
            blk = bem.block(geom, k, alpha, np.zeros(3), -np.asarray(d) * pitch, d == (0, 0, 0), rows=rows)
            acc += x[:, j, :] @ blk.T
        near_val[i] = dict(zip(rows, acc.T))
    # far field: local expansion of every listed cell, then U0 at the listed elements
    loc = {i: np.zeros((R, V0.shape[0]), dtype=np.complex128) for i in cells}
    if far:
        m = x @ V0.T                                            # [R, C, p]
        for s in range(0, len(far), chunk):
            ds = far[s:s + chunk]
            K = fmm.m2l(np.asarray(ds, dtype=np.float64) * pitch[None, :], k, order)
            for t, d in enumerate(ds):
                for i in cells:
                    j = source(i, d)
                    if j is not None:
                        loc[i] += m[:, j, :] @ K[t].T
    out = np.zeros((R, len(dofs)), dtype=np.complex128)
    for s, dof in enumerate(dofs):
        i, a = divmod(dof, n)
        out[:, s] = near_val[i][a] + loc[i] @ U0[a]
    return out


class RowSample:
    """The O2 apply on a bounded sample of one lattice, for timing the oracle:
    near field for a subset of collocation rows of every cell (rows of every S_d
    integrated once), far field (S2M for every cell, M2L chain and L2T) for a
    subset of target cells.  Scaling the two parts by n/len(rows) and
    C/len(cells) estimates the time of a full block-by-block apply."""

    def __init__(self, vertices, triangles, lattice, k, order, alpha, rows, cells, near_radius=(1, 1, 1)):
        self.grid = tuple(lattice.grid)
        self.n = int(np.asarray(triangles).shape[0])
        self.rows = np.asarray(rows)
        self.cells = np.asarray(cells)
        geom = bem.element_geometry(vertices, triangles)
        pitch = np.asarray(lattice.pitch)
        self.near = bem.near_offsets(self.grid, near_radius)
        self.S = {d: bem.block(geom, k, alpha, np.zeros(3), -np.asarray(d) * pitch, d == (0, 0, 0), rows=self.rows)
                  for d in self.near}
        self.V0 = fmm.p2m(vertices, triangles, k, order)
        self.U0 = fmm.l2p(vertices, triangles, k, order, alpha)
        self.far = far_offsets(self.grid, self.near)
        Ks = fmm.m2l(np.asarray(self.far, dtype=np.float64) * pitch[None, :], k, order) if self.far else []
        self.K = {d: Ks[i] for i, d in enumerate(self.far)}
        self._pairs = {d: pairs(self.grid, d) for d in self.near + self.far}

    def near_rows(self, x):
        """[R, C, len(rows)] = sampled rows of sum_d S_d x_{i-d} for every cell."""
        y = np.zeros((x.shape[0], x.shape[1], self.rows.size), dtype=np.complex128)
        for d in self.near:
            t, s = self._pairs[d]
            y[:, t, :] += x[:, s, :] @ self.S[d].T
        return y

    def far_cells(self, x):
        """[R, len(cells), n] = U0 sum_j K_{i-j} V0 x_j at the sampled target cells."""
        m = x @ self.V0.T
        want = set(int(c) for c in self.cells)
        loc = np.zeros((x.shape[0], x.shape[1], m.shape[2]), dtype=np.complex128)
        for d in self.far:
            t, s = self._pairs[d]
            keep = np.array([ti in want for ti in t], dtype=bool)
            if keep.any():
                loc[:, t[keep], :] += m[:, s[keep], :] @ self.K[d].T
        return loc[:, self.cells, :] @ self.U0.T
