"""Pins for oracle.operator (O2) and oracle.bem dense assembly (O1):
translation invariance, brute force block-by-block vs dense, truncation
convergence O2 -> O1, and the near-set size of the paper's 2-D example."""
import numpy as np
import pytest

from oracle import bem, operator as op
from workloads import icosphere, Lattice
from workloads.rng import random_complex


@pytest.fixture(scope="module")
def small():
    v, t = icosphere(1, 0.1)
    lat = Lattice((3, 3, 1), (0.3, 0.3, 0.3))
    k = 2 * np.pi * 800.0 / 343.0
    return v, t, lat, k, -1j / k


def test_near_set_sizes():
    # Sec. 3.3: with the unit-cell boxes and this admissibility, 2-D periodicity has 9 unique near blocks
    assert len(bem.near_offsets((5, 5, 1))) == 9
    assert len(bem.near_offsets((4, 1, 1))) == 3
    assert len(bem.near_offsets((40, 2, 8))) == 27
    far = op.far_offsets((5, 5, 1), bem.near_offsets((5, 5, 1)))
    assert len(far) == 9 * 9 - 9  # (2Mx-1)(2My-1) unique offsets of the Toeplitz structure (Sec. 2.2) minus near


def test_translation_invariance(small):
    # O1 blocks integrated from absolute coordinates equal S_d computed once (Sec. 2.2, 3.2)
    v, t, lat, k, a = small
    A = bem.dense_exact(v, t, lat, k, a)
    S = bem.near_blocks(v, t, lat, k, a)
    n = t.shape[0]
    g = op.grid_coords(lat.grid)
    for i in range(lat.n_cells):
        for j in range(lat.n_cells):
            d = tuple(int(x) for x in g[i] - g[j])
            if d in S:
                blk = A[i * n:(i + 1) * n, j * n:(j + 1) * n]
                assert np.abs(blk - S[d]).max() <= 1e-13 * np.abs(S[d]).max()


def test_block_by_block_equals_dense(small):
    v, t, lat, k, a = small
    F = op.FMPBEM(v, t, lat, k, 6, a)
    A = F.dense()
    x = random_complex((2, F.n_cells * F.n), 1)
    y = F.matvec(x)
    ref = x @ A.T
    assert np.linalg.norm(y - ref) <= 1e-14 * np.linalg.norm(ref)
    for dof in (0, 37, 5 * F.n + 3):
        assert np.allclose(F.row(dof), A[dof], rtol=0, atol=1e-15 * np.abs(A).max())


def test_truncation_converges_to_exact(small):
    v, t, lat, k, a = small
    A1 = bem.dense_exact(v, t, lat, k, a)
    x = random_complex(lat.n_cells * t.shape[0], 2)
    ref = A1 @ x
    errs = []
    for nt in (2, 4, 6, 8):
        F = op.FMPBEM(v, t, lat, k, nt, a)
        errs.append(np.linalg.norm(F.matvec(x) - ref) / np.linalg.norm(ref))
    assert all(errs[i + 1] < 0.3 * errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-5


def test_all_near_is_pbem(small):
    # with every offset in the near set, O2 is the exact periodic BEM, equal to O1 (Sec. 4: BEM and
    # PBEM agree up to round-off)
    v, t, lat, k, a = small
    F = op.FMPBEM(v, t, lat, k, 2, a, near_radius=(2, 2, 0))
    assert F.far == []
    A1 = bem.dense_exact(v, t, lat, k, a)
    x = random_complex(lat.n_cells * t.shape[0], 3)
    assert np.linalg.norm(F.matvec(x) - A1 @ x) <= 1e-13 * np.linalg.norm(A1 @ x)


def test_sampled_apply_matches_blocks(small):
    # the row-by-row sampler used at full lattice sizes agrees with the block-by-block apply
    v, t, lat, k, a = small
    F = op.FMPBEM(v, t, lat, k, 4, a)
    x = random_complex((2, lat.n_cells, t.shape[0]), 9)
    y = F.matvec(x).reshape(2, -1)
    dofs = [0, 17, 80 * 4 + 5, 80 * 8 + 79]
    ys = op.sampled_apply(v, t, lat, k, 4, a, x, dofs)
    assert np.abs(ys - y[:, dofs]).max() <= 1e-13 * np.abs(y).max()
