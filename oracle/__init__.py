"""Plain, slow FP64 CPU oracle for the high-order hexahedral operator path.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product path
(the HIP library and its Python binding) never imports, calls or links it, and
this package imports nothing from the product path: the two share only the
seeded input generators of ``paper_2109_04996_amd.inputs``, which hold no
arithmetic of the method.

What it computes, and from which passage of the paper (Kolev et al., "Efficient
Exascale Discretizations: High-Order Finite Element Methods", 2021):

* ``quadrature`` -- 1D Gauss-Legendre and Gauss-Lobatto-Legendre rules and
  C0 Lagrange tables (Benchmarks section: Q_p elements, Gauss rule with
  q = p+2 points for BP1-BP4, integration on the GLL nodes for BP5-BP6).
* ``fem`` -- trilinear brick geometry, dense element matrices by direct
  quadrature of the stiffness and mass entries A_ij = int grad phi_i . grad
  phi_j, B_ij = int phi_i phi_j (Benchmarks section), assembled into the global
  sparse matrix that the matrix-free method never forms (libCEED section,
  operator decomposition G^T B^T D B G: the assembled matrix is its exact
  value).
* ``solvers`` -- Jacobi-preconditioned CG on the Dirichlet-masked system
  (Benchmarks section: CG solves of (alpha A + beta B) u = B f with
  homogeneous Dirichlet conditions; Nekbone's diagonal preconditioner in the
  Miniapps section), a direct solve, and a Chebyshev polynomial
  preconditioner (not in the paper; textbook Chebyshev acceleration).
* ``mlp`` -- FP64 forward/backward of a two-layer tanh network (not in the
  paper; checked by finite differences).

Every pin of these functions lives in ``tests/test_oracle_*.py``.
"""
