"""FP64 CPU oracle for the matrix-free Neo-Hookean operator and its p-multigrid solver.

TEST INFRASTRUCTURE ONLY.  This package exists so that tests, the smoke check and the
benchmark's CPU-baseline leg can compare the HIP path against a plain, slow, obviously
correct implementation.  No product code imports it, and it imports nothing from the
product package: both sides receive the same arrays from the seeded input generators.

Design rules followed here (each function also cites the passage it implements):

* numpy float64 throughout; a library primitive (``inv``, ``det``, ``eigh``, sparse
  products, ``leggauss``) may serve as a step;
* naive quadrature: dense 3D element basis matrices built by explicit Kronecker loops,
  no sum factorisation and no collocated derivative;
* the constitutive law in its textbook first-Piola form ``P(F)`` and the tangent
  ``dP/dF``; the GPU path uses the paper's current-configuration Kirchhoff form, so the
  two are algebraically independent;
* multigrid transfer from its plain definition (evaluate the coarse finite-element
  function at fine nodes) and coarse operators from the Galerkin triple product.

Modules: :mod:`oracle.basis` (1D/3D tabulation), :mod:`oracle.fem` (geometry, residual,
tangent, energy, adjoint, assembly), :mod:`oracle.mg` (transfer, smoother, eigenvalue
estimate, V-cycle, Krylov and Newton drivers).
"""
