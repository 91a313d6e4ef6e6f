"""FP64 CPU oracle for the two-level Schwarz coarse solver — TEST INFRASTRUCTURE.

This package is a plain, slow, obviously-correct NumPy/SciPy statement of what the
GPU library computes, written from the paper (Ratnayaka, Fischer, Olson, "Coarse
Solvers for Exascale Solution of Poisson Problems"), Secs. 3 and 4. Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it;
the product path (the HIP library and its binding) never does, and the two share
no code. Every function cites the passage it follows.

Modules
  fem       Q1 element matrices (2x2x2 Gauss) and the assembly A = Q^T A_L Q.
  schwarz   overlapping subdomains, Boolean restrictions R_p, exact local solves.
  reduced   box grid, element-centroid cell interpolation J = W Q^T J_L S,
            cell-assembled A_r (eq. Aij), compression of unused box vertices;
            also the standard vertex-based J with Galerkin A_r = J^T A J.
  precond   additive two-level Schwarz, eq. (asm); the symmetrised hybrid.
  pcg       preconditioned conjugate gradients.
  problem   glue: one call from a mesh to an assembled preconditioner and solve.

Pins: see tests/test_oracle_*.py. Parity unpinned: the iteration counts on the
synthetic workloads (the paper prints none for them); they are compared between
oracle and GPU only.
"""
from . import fem, schwarz, reduced, precond, pcg, problem  # noqa: F401
