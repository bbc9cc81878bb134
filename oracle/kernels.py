"""Free-space Helmholtz Green's function and its normal derivatives (oracle).

Time convention e^{-i w t}, G(x, y) = e^{ikR} / (4 pi R), R = |x - y|
(Sec. 2.1, eq. (green3dFull)).  With r = x - y and E = e^{ikR}/(4 pi):

    dG/dn_y        =  E (1 - ikR) (r.n_y) / R^3
    dG/dn_x        = -E (1 - ikR) (r.n_x) / R^3
    d2G/dn_x dn_y  =  E [ (1 - ikR)(n_x.n_y) / R^3 - (3 - 3ikR - k^2R^2)(r.n_x)(r.n_y) / R^5 ]

which follow from dG/dR = E (ikR - 1)/R^2 and the chain rule (r = x - y, so
grad_y R = -r/R and grad_x R = r/R).  These enter the CBIE (eq. (cbie)), the
HBIE (eq. (hbie)) and their Burton-Miller combination (eq. (bm)).
"""
from __future__ import annotations

import numpy as np

FOUR_PI = 4.0 * np.pi


def green(x, y, k):
    r = np.asarray(x) - np.asarray(y)
    R = np.linalg.norm(r, axis=-1)
    return np.exp(1j * k * R) / (FOUR_PI * R)


def dgreen_dny(x, y, ny, k):
    r = np.asarray(x) - np.asarray(y)
    R = np.linalg.norm(r, axis=-1)
    E = np.exp(1j * k * R) / FOUR_PI
    return E * (1.0 - 1j * k * R) * (r * ny).sum(-1) / R ** 3


def dgreen_dnx(x, y, nx, k):
    r = np.asarray(x) - np.asarray(y)
    R = np.linalg.norm(r, axis=-1)
    E = np.exp(1j * k * R) / FOUR_PI
    return -E * (1.0 - 1j * k * R) * (r * nx).sum(-1) / R ** 3


def d2green_dnxdny(x, y, nx, ny, k):
    r = np.asarray(x) - np.asarray(y)
    R = np.linalg.norm(r, axis=-1)
    E = np.exp(1j * k * R) / FOUR_PI
    ikr = 1j * k * R
    rnx = (r * nx).sum(-1)
    rny = (r * ny).sum(-1)
    nxny = (np.asarray(nx) * np.asarray(ny)).sum(-1)
    return E * ((1.0 - ikr) * nxny / R ** 3
                - (3.0 - 3.0 * ikr - (k * R) ** 2) * rnx * rny / R ** 5)


def bm_kernel(x, y, nx, ny, k, alpha):
    """Kernel of the Burton-Miller double-layer part, dG/dn_y + alpha d2G/dn_x dn_y
    (eq. (bm)); alpha = 0 gives the CBIE kernel (eq. (cbie))."""
    out = dgreen_dny(x, y, ny, k)
    if alpha != 0:
        out = out + alpha * d2green_dnxdny(x, y, nx, ny, k)
    return out
