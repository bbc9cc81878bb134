"""FP64 CPU oracle for the fast multipole periodic BEM (FMPBEM) operator and solve.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(``paper_2201_12050_amd``) never does, and shares no code with it.

Contents (paper sections in brackets):
  quadrature  Gauss-Legendre nodes by Newton's method; Duffy-collapsed triangle rules
  kernels     Green's function G and its normal derivatives [Sec. 2.1, eq. (green3dFull), (hbie), (bm)]
  bem         collocation entries, near-field blocks S_d, dense exact BEM (O1), incident fields [Sec. 2.1-2.2];
              pressure at points of the fluid, insertion loss [eq. (cbie) with c = 1, eq. (insertionloss)]
  specfun     spherical Bessel/Hankel (SciPy), harmonics, Wigner 3j (Racah, exact integers)
  fmm         P2M (V0), L2P (U0), M2L (K_d) operators [Sec. 3.1, Appendix A]
  operator    FMPBEM operator S + U K V applied block by block, no FFT (O2) [Sec. 3.2]
  solve       dense LU and restarted GMRES [Sec. 3.5, Sec. 4]
  halfspace   half-space Green's function: image blocks, image multipole chain, incident fields
              and field evaluation with the image terms [eq. (green3dHalf), Sec. 2.3, Sec. 3.4]
  mie         Mie series for a rigid sphere (analytic pin, not from the paper)

Every function here is pinned by a ``-m "not gpu"`` test against closed forms,
library special cases, finite differences, invariants or brute force; see the
tests named ``tests/test_oracle_*.py``.
"""
