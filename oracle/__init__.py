"""CPU oracle for the finite-element Kohn-Sham H.X hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, tables or
helpers with the HIP library under ``paper_2512_08571_amd/``.

What it computes, and how (all in float64 / complex128):

* ``basis``      1D Gauss-Lobatto-Legendre nodes and weights, Gauss-Legendre
                 quadrature, Lagrange shape functions and their *direct*
                 derivatives (product rule) -- Sec. 2.2, eqn FEdiscr.
* ``mesh``       periodic (or open) parallelepiped mesh, affine cell map,
                 the cell-to-DoF map Q^(e) with the periodic wrap playing the
                 role of the constraint matrix C -- Sec. 3, eqn HX.
* ``operator``   cell matrices T, L, G, K, M by explicit 3D quadrature of the
                 integrals in eqn Hloc / HlocIntegral (no sum factorisation,
                 no collocation derivative), assembly into global sparse
                 matrices, the lumped GLL mass D, the nonlocal projector
                 matrix of eqn Vnonloc, and H.X by (i) the assembled sparse
                 product, (ii) the cell-matrix route, (iii) row sampling.
* ``projectors`` the analytic projector functions (one reading of the paper,
                 which leaves their form to the pseudopotential).
* ``eigen``      the residual Chebyshev filter (Alg. 4), Rayleigh-Ritz
                 (Alg. 3), Lanczos spectral bounds and the outer driver.
* ``flops``      the paper's operation-count model (eqns flopRealMF,
                 flopComplexMF, flopRealCM, flopComplexCM).

Parity pins: every function here is checked in ``tests/test_oracle_*.py``
against closed forms, invariants, special cases or brute force (see the
header of each module).  Nothing in the oracle is "parity unpinned".
"""
