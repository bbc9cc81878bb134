"""Pins for oracle.fmm: the P2M -> M2L -> L2P chain reproduces the exact kernels
(addition theorem), converges geometrically in n_t, is reciprocal, and the
printed power of i in the M2L coefficient fails (regression guard)."""
import numpy as np
import pytest

from oracle import fmm, kernels, specfun

K1K = 2 * np.pi * 1000.0 / 343.0
FAC = lambda nt: np.array([(2 * n + 1) for n in range(nt + 1) for _ in range(2 * n + 1)], dtype=np.float64)


def _points(rng, radius, count):
    v = rng.normal(size=(count, 3))
    return v * (radius / np.linalg.norm(v, axis=1, keepdims=True))


def _chain(x_loc, y_loc, D, k, nt, nx=None, ny=None, K=None):
    """Far-field value of the kernel for target x_loc (relative to its cell centre)
    and source y_loc (relative to the source centre), centres D apart."""
    if K is None:
        K = fmm.m2l(D[None], k, nt)[0]
    if ny is None:
        M = np.conj(fmm.regular(y_loc[None], k, nt))[0]
    else:
        M = (fmm.grad_conj_regular(y_loc[None], k, nt)[0] * ny).sum(-1)
    if nx is None:
        Ic = np.conj(fmm.regular(x_loc[None], k, nt))[0]
    else:
        Ic = (fmm.grad_conj_regular(x_loc[None], k, nt)[0] * nx).sum(-1)
    return 1j * k / (4 * np.pi) * (FAC(nt) * Ic) @ (K @ M)


OFFSETS = [np.array([0.6, 0.0, 0.0]), np.array([0.6, 0.3, 0.0]), np.array([0.9, -0.6, 0.0]),
           np.array([0.0, 0.0, 0.6]), np.array([0.6, 0.3, 0.3])]


@pytest.mark.parametrize("kind", ["G", "dG/dny", "d2G/dnxdny"])
def test_chain_reproduces_kernels(kind):
    rng = np.random.default_rng(21)
    nt = 10
    worst = 0.0
    for D in OFFSETS:
        K = fmm.m2l(D[None], K1K, nt)[0]
        for _ in range(4):
            x = _points(rng, 0.1, 1)[0]
            y = _points(rng, 0.1, 1)[0]
            nx = _points(rng, 1.0, 1)[0]
            ny = _points(rng, 1.0, 1)[0]
            if kind == "G":
                ex = kernels.green(x + D, y, K1K)
                ap = _chain(x, y, D, K1K, nt, K=K)
            elif kind == "dG/dny":
                ex = kernels.dgreen_dny(x + D, y, ny, K1K)
                ap = _chain(x, y, D, K1K, nt, ny=ny, K=K)
            else:
                ex = kernels.d2green_dnxdny(x + D, y, nx, ny, K1K)
                ap = _chain(x, y, D, K1K, nt, nx=nx, ny=ny, K=K)
            worst = max(worst, abs(ap - ex) / abs(ex))
    assert worst < 1e-5  # truncation error of n_t = 10 at 1 kHz, closest far offset


def test_chain_converges_geometrically():
    rng = np.random.default_rng(3)
    D = OFFSETS[1]
    pts = [(_points(rng, 0.1, 1)[0], _points(rng, 0.1, 1)[0]) for _ in range(6)]
    errs = []
    for nt in (2, 4, 6, 8, 10):
        e = max(abs(_chain(x, y, D, K1K, nt) - kernels.green(x + D, y, K1K)) / abs(kernels.green(x + D, y, K1K))
                for x, y in pts)
        errs.append(e)
    assert all(errs[i + 1] < 0.2 * errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-6


def test_printed_power_of_i_fails():
    # Using i^{n'-n+l} instead of i^{n-n'+l} multiplies K_d entrywise by (-1)^{n+n'}.
    rng = np.random.default_rng(4)
    nt = 8
    D = OFFSETS[0]
    K = fmm.m2l(D[None], K1K, nt)[0]
    sgn = np.array([(-1.0) ** n for n in range(nt + 1) for _ in range(2 * n + 1)])
    Kp = sgn[:, None] * K * sgn[None, :]
    x, y = _points(rng, 0.1, 1)[0], _points(rng, 0.1, 1)[0]
    ex = kernels.green(x + D, y, K1K)
    assert abs(_chain(x, y, D, K1K, nt, K=K) - ex) < 1e-4 * abs(ex)
    assert abs(_chain(x, y, D, K1K, nt, K=Kp) - ex) > 0.1 * abs(ex)


def test_m2l_reciprocity():
    nt = 8
    sgn = np.array([(-1.0) ** n for n in range(nt + 1) for _ in range(2 * n + 1)])
    for D in OFFSETS:
        Kp, Km = fmm.m2l(np.stack([D, -D]), K1K, nt)
        assert np.abs(Km - sgn[:, None] * Kp * sgn[None, :]).max() < 1e-13 * np.abs(Kp).max()
    # exact reciprocity of the chain: x <- y via +D equals y <- x via -D
    rng = np.random.default_rng(9)
    x, y = _points(rng, 0.1, 1)[0], _points(rng, 0.1, 1)[0]
    D = OFFSETS[2]
    a = _chain(x, y, D, K1K, nt)
    b = _chain(y, x, -D, K1K, nt)
    assert abs(a - b) < 1e-14 * abs(a)


def test_m2l_monopole_term():
    # K_d[(0,0),(0,0)] = O_0^0(D) = h_0(k|D|): the l = 0 term that strict bounds would drop
    D = OFFSETS[0]
    K = fmm.m2l(D[None], K1K, 3)[0]
    assert np.isclose(K[0, 0], specfun.sph_h(0, K1K * np.linalg.norm(D)), rtol=1e-14)
