"""Single-level multipole operators of the FMPBEM (oracle; test infrastructure).

Expansion of G (Sec. 3.1, eq. (greenFMM)), with the argument k|x| in the
radial functions (eq. (Onm) prints |x|; the expansion only converges with the
wavenumber included):

    G(x, y) ~ (ik/4pi) sum_n (2n+1) sum_m O_n^m(x - y_c) conj(I_n^m(y - y_c)),
    O_n^m(v) = h_n(k|v|) Y_n^m(v/|v|),   I_n^m(v) = j_n(k|v|) Y_n^m(v/|v|).

Operators (Appendix A), every cell using the same matrices (Sec. 3.2):
  V0 (P2M, eq. (p2m)):  V0[(n,m), b] = int_{Delta_b} d/dn_y conj(I_n^m(y - c)) dA(y)
                        (8 x 8 Duffy rule on each element)
  U0 (L2P, eq. (l2p)):  U0[a, (n,m)] = (ik/4pi)(2n+1) [conj(I_n^m(x_a - c))
                                        + alpha d/dn_x conj(I_n^m(x_a - c))]
                        (the alpha term carries the hypersingular kernel of eq. (bm))
  K_d (M2L, eq. (m2l)): K_d[(n,m),(n',m')] = (2n'+1)(-1)^{m+m'}
                          sum_l W_{n',n,m',m,l} O_l^{m+m'}(d*pitch)
    with W = (2l+1) i^{n-n'+l} (n n' l; 0 0 0)(n n' l; m m' -m-m')  (eq. (wigner))
    and l over max(|m+m'|, |n-n'|) <= l <= n+n', n+n'-l even.

Multilevel translations (Appendix A, eqs. (m2m), (l2l); used by the FMPBEM2
near field of Sec. 3.3):
  T(b) (M2M, eq. (m2m)): moments about y_c' from moments about y_c, b = y_c - y_c'
      T[(n,m),(n',m')] = (2n'+1)(-1)^{m'} sum_l W_{n,n',m,-m',l} I_l^{m'-m}(b)
      (eq. (m2m) with its summation index m' renamed to -m'); it is the
      regular addition theorem conj(I_n^m(a + b)) = sum T[(n,m),(n',m')] conj(I_n'^m'(a)).
  L2L: local coefficients about x_c' from those about x_c, b = x_c' - x_c
      L'(n,m) = (-1)^m sum_{n',m'} (2n'+1) sum_l W_{n',n,m',-m,l} I_l^{m-m'}(b) L(n',m'),
      i.e. (2n+1) L'(n,m) = sum (2n'+1) T[(n',m'),(n,m)](b) L(n',m'): the expansion of
      eq. (l2p) re-centred with the same addition theorem.
  Both truncate the source order at n_t (exact as the source order grows).

Readings of the printed formulas (each checked against the exact kernel by
the addition-theorem tests): the bounds on l are inclusive (the printed strict
bounds leave the monopole term n = n' = 0 empty), the power of i in W is
n - n' + l (the printed n' - n + l does not reproduce G), and the harmonics
carry the (-1)^m phase stated in ``specfun``.  The same power reading holds in
eq. (m2m) (W_{n,n',...} takes i^{n'-n+l}); in eq. (l2l) the second row of the
second 3j symbol reads (-m, m', m-m'), matching the order m - m' of I_l (the
printed (m, m', -m-m') pairs it with I_l^{-m-m'}).
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
import scipy.sparse as sp

from . import specfun
from .quadrature import duffy_points

FOUR_PI = 4.0 * np.pi


def n_coeffs(order: int) -> int:
    return (order + 1) ** 2


def regular(v, k, order):
    """I_n^m(v) for all (n, m): [..., p]."""
    r, ct, phi = specfun.spherical_coords(v)
    Y = specfun.harmonics(ct, phi, order)
    out = np.empty_like(Y)
    for n in range(order + 1):
        jn = specfun.sph_j(n, k * r)
        out[..., n * n:(n + 1) * (n + 1)] = jn[..., None] * Y[..., n * n:(n + 1) * (n + 1)]
    return out


def singular(v, k, order):
    """O_n^m(v) for all (n, m): [..., p]."""
    r, ct, phi = specfun.spherical_coords(v)
    Y = specfun.harmonics(ct, phi, order)
    out = np.empty_like(Y)
    for n in range(order + 1):
        hn = specfun.sph_h(n, k * r)
        out[..., n * n:(n + 1) * (n + 1)] = hn[..., None] * Y[..., n * n:(n + 1) * (n + 1)]
    return out


def grad_conj_regular(v, k, order):
    """Gradient of conj(I_n^m(v)) with respect to v: [..., p, 3] (spherical-coordinate formula)."""
    v = np.asarray(v, dtype=np.float64)
    r, ct, phi = specfun.spherical_coords(v)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    if np.any((st == 0) & (r > 0)):
        raise ValueError("point on the polar axis")
    Y, dY = specfun.harmonics(ct, phi, order, with_dtheta=True)
    cp, sp_ = np.cos(phi), np.sin(phi)
    rhat = np.stack([st * cp, st * sp_, ct], -1)
    that = np.stack([ct * cp, ct * sp_, -st], -1)
    phat = np.stack([-sp_, cp, np.zeros_like(cp)], -1)
    p = n_coeffs(order)
    g = np.zeros(v.shape[:-1] + (p, 3), dtype=np.complex128)
    for n in range(order + 1):
        jn = specfun.sph_j(n, k * r)
        jd = specfun.sph_jd(n, k * r)
        for m in range(-n, n + 1):
            i = specfun.idx(n, m)
            gr = k * jd * Y[..., i]
            gt = jn / r * dY[..., i]
            gp = jn / (r * st) * 1j * m * Y[..., i]
            grad = gr[..., None] * rhat + gt[..., None] * that + gp[..., None] * phat
            g[..., i, :] = np.conj(grad)
    return g


def p2m(vertices, triangles, k, order, q: int = 8, center=None):
    """V0 [p, n]: P2M moments of each element for unit density (eq. (p2m)), about
    ``center``: one point [3] for every element (the cell centre, the origin, by default)
    or one per element [n, 3]."""
    v = np.asarray(vertices, dtype=np.float64)
    t = np.asarray(triangles)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    if center is not None:
        cen = np.asarray(center, dtype=np.float64)
        a, b, c = a - cen, b - cen, c - cen
    nrm = np.cross(b - a, c - a)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    out = np.zeros((n_coeffs(order), a.shape[0]), dtype=np.complex128)
    step = 256  # elements per vectorised batch
    for s in range(0, a.shape[0], step):
        e = slice(s, s + step)
        pts, w = duffy_points(a[e], b[e], c[e], q)           # [ne, q*q, 3], [ne, q*q]
        g = grad_conj_regular(pts, k, order)                 # [ne, q*q, p, 3]
        dn = (g * nrm[e][:, None, None, :]).sum(-1)          # [ne, q*q, p]
        out[:, e] = (dn * w[..., None]).sum(1).T
    return out                                               # [p, n]


def l2p(vertices, triangles, k, order, alpha, center=None):
    """U0 [n, p]: local-to-collocation-point operator incl. the Burton-Miller term (eq. (l2p)),
    local expansion about ``center`` (the origin by default)."""
    v = np.asarray(vertices, dtype=np.float64)
    if center is not None:
        v = v - np.asarray(center, dtype=np.float64)[None, :]
    t = np.asarray(triangles)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    nrm = np.cross(b - a, c - a)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    x = (a + b + c) / 3.0
    Ic = np.conj(regular(x, k, order))                       # [n, p]
    out = Ic.copy()
    if alpha != 0:
        g = grad_conj_regular(x, k, order)                   # [n, p, 3]
        out = out + alpha * (g * nrm[:, None, :]).sum(-1)
    fac = np.array([(2 * n + 1) for n in range(order + 1) for _ in range(2 * n + 1)], dtype=np.float64)
    return (1j * k / FOUR_PI) * out * fac[None, :]


@lru_cache(maxsize=None)
def m2l_table(order: int):
    """Sparse map T [(p*p), (2*order+1)^2] with K_d.ravel() = T @ O(d), from eq. (m2l)-(wigner)."""
    rows, cols, vals = [], [], []
    p = n_coeffs(order)
    for n in range(order + 1):
        for m in range(-n, n + 1):
            for n2 in range(order + 1):
                for m2 in range(-n2, n2 + 1):
                    mu = m + m2
                    lo = max(abs(mu), abs(n - n2))
                    for l in range(lo, n + n2 + 1):
                        if (n + n2 - l) % 2:
                            continue
                        w = (2 * l + 1) * specfun.wigner3j(n, n2, l, 0, 0, 0) * specfun.wigner3j(n, n2, l, m, m2, -mu)
                        if w == 0.0:
                            continue
                        coef = (2 * n2 + 1) * (-1.0) ** (m + m2) * w * (1j ** ((n - n2 + l) % 4))
                        rows.append(specfun.idx(n, m) * p + specfun.idx(n2, m2))
                        cols.append(specfun.idx(l, mu))
                        vals.append(coef)
    return sp.csr_matrix((np.array(vals, dtype=np.complex128), (rows, cols)),
                         shape=(p * p, (2 * order + 1) ** 2))


def m2l(offsets_xyz, k, order):
    """K_d [len, p, p] for centre offsets D = x_c - y_c (target minus source), eq. (m2l)."""
    D = np.atleast_2d(np.asarray(offsets_xyz, dtype=np.float64))
    O = singular(D, k, 2 * order)                           # [nd, (2nt+1)^2]
    T = m2l_table(order)
    p = n_coeffs(order)
    return np.asarray((T @ O.T).T).reshape(D.shape[0], p, p)


@lru_cache(maxsize=None)
def m2m_table(order: int, order_src: int | None = None):
    """Sparse map T [(p_t*p_s), (n_t+n_s+1)^2] with M2M(b).ravel() = T @ I(b), eq. (m2m).
    Rows (n, m) up to ``order``, columns (n', m') up to ``order_src`` (default: ``order``)."""
    ns = order if order_src is None else order_src
    rows, cols, vals = [], [], []
    ps = n_coeffs(ns)
    for n in range(order + 1):
        for m in range(-n, n + 1):
            for n2 in range(ns + 1):
                for m2 in range(-n2, n2 + 1):
                    mu = m2 - m  # order of I_l
                    for l in range(max(abs(mu), abs(n - n2)), n + n2 + 1):
                        if (n + n2 - l) % 2:
                            continue
                        # W_{n,n',m,-m',l}: (2l+1) i^{n'-n+l} (n' n l; 0 0 0)(n' n l; -m' m m'-m)
                        w = (2 * l + 1) * specfun.wigner3j(n2, n, l, 0, 0, 0) * specfun.wigner3j(n2, n, l, -m2, m, mu)
                        if w == 0.0:
                            continue
                        coef = (2 * n2 + 1) * (-1.0) ** m2 * w * (1j ** ((n2 - n + l) % 4))
                        rows.append(specfun.idx(n, m) * ps + specfun.idx(n2, m2))
                        cols.append(specfun.idx(l, mu))
                        vals.append(coef)
    return sp.csr_matrix((np.array(vals, dtype=np.complex128), (rows, cols)),
                         shape=(n_coeffs(order) * ps, (order + ns + 1) ** 2))


def m2m(shifts, k, order, order_src=None):
    """M2M [len, p_t, p_s] for b = y_c - y_c' (old centre minus new centre), eq. (m2m)."""
    ns = order if order_src is None else order_src
    b = np.atleast_2d(np.asarray(shifts, dtype=np.float64))
    Ib = regular(b, k, order + ns)
    T = m2m_table(order, order_src)
    return np.asarray((T @ Ib.T).T).reshape(b.shape[0], n_coeffs(order), n_coeffs(ns))


@lru_cache(maxsize=None)
def l2l_table(order: int, order_src: int | None = None):
    """Sparse map T [(p_t*p_s), (n_t+n_s+1)^2] with L2L(b).ravel() = T @ I(b), eq. (l2l)."""
    ns = order if order_src is None else order_src
    rows, cols, vals = [], [], []
    ps = n_coeffs(ns)
    for n in range(order + 1):
        for m in range(-n, n + 1):
            for n2 in range(ns + 1):
                for m2 in range(-n2, n2 + 1):
                    mu = m - m2  # order of I_l
                    for l in range(max(abs(mu), abs(n - n2)), n + n2 + 1):
                        if (n + n2 - l) % 2:
                            continue
                        # W_{n',n,m',-m,l}: (2l+1) i^{n-n'+l} (n n' l; 0 0 0)(n n' l; -m m' m-m')
                        w = (2 * l + 1) * specfun.wigner3j(n, n2, l, 0, 0, 0) * specfun.wigner3j(n, n2, l, -m, m2, mu)
                        if w == 0.0:
                            continue
                        coef = (2 * n2 + 1) * (-1.0) ** m * w * (1j ** ((n - n2 + l) % 4))
                        rows.append(specfun.idx(n, m) * ps + specfun.idx(n2, m2))
                        cols.append(specfun.idx(l, mu))
                        vals.append(coef)
    return sp.csr_matrix((np.array(vals, dtype=np.complex128), (rows, cols)),
                         shape=(n_coeffs(order) * ps, (order + ns + 1) ** 2))


def l2l(shifts, k, order, order_src=None):
    """L2L [len, p_t, p_s] for b = x_c' - x_c (new centre minus old centre), eq. (l2l)."""
    ns = order if order_src is None else order_src
    b = np.atleast_2d(np.asarray(shifts, dtype=np.float64))
    Ib = regular(b, k, order + ns)
    T = l2l_table(order, order_src)
    return np.asarray((T @ Ib.T).T).reshape(b.shape[0], n_coeffs(order), n_coeffs(ns))
