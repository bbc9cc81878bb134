"""Solvers (oracle; test infrastructure): dense LU and restarted GMRES.

The paper solves with GMRES to a relative tolerance (Sec. 4); restart length,
orthogonalisation and norm are not stated.  The oracle uses GMRES(m) with
modified Gram-Schmidt, Givens rotations and the relative residual
||b - A x||_2 / ||b||_2, no preconditioner.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def lu_solve(A, b):
    lu = sla.lu_factor(A)
    return sla.lu_solve(lu, b)


def gmres(matvec, b, tol=1e-12, restart=100, maxiter=2000, x0=None):
    """Returns (x, iterations, relative residual)."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        return x, 0, 0.0
    its = 0
    while its < maxiter:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            return x, its, beta / bnorm
        m = restart
        V = np.zeros((m + 1, b.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            w = matvec(V[j])
            its += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                # rotation i: [[conj(c), conj(s)], [-s, c]]
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[j] = a / den if den != 0 else 1.0
            sn[j] = bb / den if den != 0 else 0.0
            H[j, j] = np.conj(cs[j]) * a + np.conj(sn[j]) * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            j_done = j + 1
            if abs(g[j + 1]) / bnorm <= tol or its >= maxiter:
                break
        y = sla.solve_triangular(H[:j_done, :j_done], g[:j_done])
        x = x + V[:j_done].T @ y
    r = b - matvec(x)
    return x, its, np.linalg.norm(r) / bnorm
