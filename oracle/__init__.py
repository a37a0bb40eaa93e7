"""CPU oracle for the D3M factor/solve path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct NumPy/SciPy implementation of what the
method computes, written from the paper (Moshfegh & Vouvakis, "Direct Domain
Decomposition Method (D3M) for Finite Element Electromagnetic Computations",
Section II: the decomposed boundary-value problem, eq. (1), the seven-step
recipe and Algorithm 1).  Complex128 throughout.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2002_05018_amd``) and imports nothing from it; the two meet only in
the seeded input generator ``workloads``.

Modules
-------
``quad``   triangle quadrature (Gauss-Legendre on the collapsed square)
``fem``    mesh topology, Whitney element matrices, first-order ABC,
           plane-wave load, global matrix S (the undecomposed FEM system)
``ddm``    the decomposed system: subdomain matrices A_d with the Robin
           loss/gain terms, Lagrange-multiplier (LM) trees and the signed maps
           D_d, domain matrices K_D^(d) = D_d^T A_d^{-1} D_d, K and g
``bk``     dense complex-symmetric Bunch-Kaufman LDL^T (reference [bunch1977])
``block``  geometric nested dissection of the block (clique) graph, block
           symbolic factorisation and Algorithm 1 (block LDL^T with pivoting
           restricted to each diagonal block), block forward/diagonal/backward
           substitution
``d3m``    the seven steps end to end, recovery of E and the adjoint gradient

Every function with no independent pin says "parity unpinned" in its
docstring; the pins live in ``tests/test_oracle_*.py``.
"""
