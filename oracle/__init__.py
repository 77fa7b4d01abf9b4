"""Plain FP64 CPU oracle for the KIOPS φ-combination (test infrastructure only).

This package is the independent reference that the HIP library is checked
against.  It is slow on purpose, written for a reader holding the paper
(Gaudreault, Rainwater & Tokman, "KIOPS: A fast adaptive Krylov subspace
solver for exponential integators", J. Comput. Phys. 372 (2018), with its
corrigendum).  It shares no code with the HIP path and never imports it.

Only the test suite, the smoke check in ``__graft_entry__`` and the CPU
baseline leg of ``bench.py`` may import anything from here; the product path
must never route through it.

Modules:
  phi        scalar phi_k(z) of Eq. (3)
  expm       dense matrix exponential by its power series and squaring
  operators  the stencil / CSR operators applied and assembled from their data
  augmented  Theorem 1: the augmented matrix (13) and the dense exact result (14)
  spectral   exact result for constant-coefficient periodic stencils via the DFT
  arnoldi    exact-to-tolerance result for large N via full-Arnoldi Krylov
  lanczos    exact-to-tolerance result for symmetric A, one Lanczos process per term
  iop        Algorithm 2 (incomplete orthogonalization, window q)
  controller Algorithm 4 with Sections 3.5-3.6 (acceptance, step size, dimension)
  kiops      Algorithm 1 (Task II) assembled from the pieces above
"""
