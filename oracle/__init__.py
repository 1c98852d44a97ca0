"""ORACLE: plain, slow, CPU FP64 reference of the surface-multigrid V-cycle.

This package is test infrastructure.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product library (``paper_2104_13755_amd``) never imports,
links or executes anything here, and this package never imports the product.

Parts (each module cites the passage of the paper it follows):
  assemble   cotan Laplacian L and lumped mass M (A = M + t L)
  native     the plain-C pieces (successive self-parameterization, coloring)
  hierarchy  prolongations P_l, Galerkin A_{l+1} = P_l^T A_l P_l, coloring
  vcycle     multicolor Gauss-Seidel, residual, transfer, coarsest Cholesky,
             the V-cycle (Alg. V-cycle) and the solve loop (Alg. Galerkin
             Surface Multigrid Solver)
  grad       adjoint gradients of a linear loss through the solve
"""
