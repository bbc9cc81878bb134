"""Pins of the FMPBEM2 oracle (Sec. 3.3; Appendix A eqs. (m2m), (l2l)): the translations
reproduce the regular functions they re-centre (addition theorem, exact as the source
order grows), the centred P2M / L2P agree with the translations, the leaf-pair levels
agree with an explicit dual-tree traversal, and the approximated near blocks converge to
the exact ones as n_t,near grows."""
import numpy as np
import pytest

from oracle import bem, fmm, multilevel as ml
from oracle.operator import FMPBEM
from workloads import icosphere, Lattice

K = 2 * np.pi * 800 / 343.0


def _fac(order):
    return np.array([2 * n + 1 for n in range(order + 1) for _ in range(2 * n + 1)], dtype=np.float64)


def test_m2m_is_the_regular_addition_theorem():
    rng = np.random.default_rng(11)
    b = np.array([0.021, -0.013, 0.034])
    a = rng.normal(size=(24, 3)) * 0.02
    T = fmm.m2m(b, K, 5, 24)[0]
    lhs = np.conj(fmm.regular(a + b, K, 5))
    rhs = np.conj(fmm.regular(a, K, 24)) @ T.T
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(lhs).max()
    # the translation depends on the direction of b (a swapped shift fails)
    assert np.abs(T - fmm.m2m(-b, K, 5, 24)[0]).max() > 1e-3


def test_l2l_recentres_the_local_expansion():
    rng = np.random.default_rng(12)
    order, big = 5, 24
    L = rng.normal(size=fmm.n_coeffs(order)) + 1j * rng.normal(size=fmm.n_coeffs(order))
    xc2 = np.array([0.012, 0.02, -0.017])
    x = xc2 + rng.normal(size=(16, 3)) * 0.01
    f_old = (np.conj(fmm.regular(x, K, order)) * _fac(order)) @ L
    L2 = fmm.l2l(xc2, K, big, order)[0] @ L
    f_new = (np.conj(fmm.regular(x - xc2, K, big)) * _fac(big)) @ L2
    assert np.abs(f_old - f_new).max() <= 1e-13 * np.abs(f_old).max()


def test_centred_p2m_and_l2p_agree_with_the_translations():
    v, t = icosphere(1, 0.1)
    t = t[:12]
    child = np.array([0.0375, -0.0375, 0.0375])
    parent = np.array([0.075, -0.075, 0.075])
    order, big = 4, 22
    # moments about the parent from moments about the child (M2M with b = child - parent)
    direct = fmm.p2m(v, t, K, order, center=parent)
    moved = fmm.m2m(child - parent, K, order, big)[0] @ fmm.p2m(v, t, K, big, center=child)
    assert np.abs(direct - moved).max() <= 1e-12 * np.abs(direct).max()
    # local coefficients about the parent evaluated at the child's points: L2P about the
    # parent = L2P about the child after L2L with b = child - parent
    alpha = -1j / K
    L = np.random.default_rng(5).normal(size=fmm.n_coeffs(order)) + 0j
    at_parent = fmm.l2p(v, t, K, order, alpha, center=parent) @ L
    at_child = fmm.l2p(v, t, K, big, alpha, center=child) @ (fmm.l2l(child - parent, K, big, order)[0] @ L)
    assert np.abs(at_parent - at_child).max() <= 1e-12 * np.abs(at_parent).max()


def _traverse(tree, d):
    """Explicit dual-tree descent from the two cell boxes: {(leaf a, leaf b): level} of the
    translations, and the set of leaf pairs left near on the finest level."""
    L = tree.levels
    occupied = [set(map(tuple, tree.coords(l))) for l in range(L + 1)]
    leaves = tree.leaves()
    far, near = {}, set()

    def below(box, lev):
        return [c for c in leaves if tuple(np.asarray(c) >> (L - lev)) == box]

    def visit(a, b, lev):
        delta = np.asarray(a) - np.asarray(b) + np.asarray(d) * (1 << lev)
        if np.max(np.abs(delta)) >= 2:
            for ca in below(a, lev):
                for cb in below(b, lev):
                    assert (ca, cb) not in far
                    far[(ca, cb)] = lev
            return
        if lev == L:
            near.add((a, b))
            return
        for ca in occupied[lev + 1]:
            if tuple(np.asarray(ca) >> 1) != a:
                continue
            for cb in occupied[lev + 1]:
                if tuple(np.asarray(cb) >> 1) == b:
                    visit(ca, cb, lev + 1)

    visit((0, 0, 0), (0, 0, 0), 0)
    return far, near


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_interaction_levels_match_a_dual_tree_descent(levels):
    v, t = icosphere(1, 0.1)
    tree = ml.CellTree(v, t, (0.3, 0.3, 0.3), levels)
    leaves = list(tree.leaves())
    for d in bem.near_offsets((3, 3, 1)):
        far, near = _traverse(tree, d)
        assert len(far) + len(near) == len(leaves) ** 2       # every leaf pair exactly once
        for a in leaves:
            for b in leaves:
                lev = ml.interaction_level(tree, a, b, d)
                assert lev == far.get((a, b)), (d, a, b)
                assert (lev is None) == ((a, b) in near)


def test_levels_zero_keeps_the_exact_blocks():
    v, t = icosphere(1, 0.1)
    lat = Lattice((3, 3, 1), (0.3, 0.3, 0.3))
    S = bem.near_blocks(v, t, lat, K, -1j / K)
    A = ml.approx_blocks(v, t, lat, K, -1j / K, 0, 4, exact=S)
    for d in S:
        assert np.array_equal(A[d], S[d])


def test_near_blocks_converge_to_the_exact_ones():
    v, t = icosphere(2, 0.1)
    lat = Lattice((3, 3, 1), (0.3, 0.3, 0.3))
    alpha = -1j / K
    S = bem.near_blocks(v, t, lat, K, alpha)
    errs = []
    for nt in (2, 4, 6, 8):
        A = ml.approx_blocks(v, t, lat, K, alpha, 2, nt, exact=S)
        errs.append(max(np.linalg.norm(A[d] - S[d]) / np.linalg.norm(S[d]) for d in S))
    # geometric convergence in n_t,near (measured 0.128, 0.0113, 0.0027, 0.00069)
    assert all(e2 < e1 / 3 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3, errs


def test_fmpbem2_matvec_is_its_dense_operator():
    v, t = icosphere(1, 0.1)
    lat = Lattice((4, 3, 1), (0.3, 0.3, 0.3))
    F = ml.FMPBEM2(v, t, lat, K, 4, -1j / K, 2, 4)
    x = np.random.default_rng(3).normal(size=(2, lat.n_cells * 80)) + 0j
    y = F.matvec(x)
    yd = x @ F.dense().T
    assert np.abs(y - yd).max() <= 1e-12 * np.abs(yd).max()
    # the far field is the FMPBEM's, only the near blocks differ
    F1 = FMPBEM(v, t, lat, K, 4, -1j / K)
    assert F.K.keys() == F1.K.keys() and all(np.array_equal(F.K[d], F1.K[d]) for d in F1.K)
