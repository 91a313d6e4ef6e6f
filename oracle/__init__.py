"""FP64 CPU oracle for the two-level Schwarz coarse solver — TEST INFRASTRUCTURE.

This package is a plain, slow, obviously-correct NumPy/SciPy statement of what the
GPU library computes, written from the paper (Ratnayaka, Fischer, Olson, "Coarse
Solvers for Exascale Solution of Poisson Problems"), Secs. 3 and 4. Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it;
the product path (the HIP library and its binding) never does, and the two share
no code. Every function cites the passage it follows.

Modules
  fem       Q1 element matrices (2x2x2 Gauss) and the assembly A = Q^T A_L Q.
  schwarz   overlapping subdomains, Boolean restrictions R_p, exact local solves,
            and the inexact ones (k steps of Jacobi-preconditioned CG per
            subdomain, Sec. 6.3).
  reduced   box grid, element-centroid cell interpolation J = W Q^T J_L S,
            cell-assembled A_r (eq. Aij), compression of unused box vertices;
            also the standard vertex-based J with Galerkin A_r = J^T A J.
  precond   additive two-level Schwarz, eq. (asm); its local and reduced parts
            alone; the hybrid of eqs. (asm1)-(asm2) as written; the
            symmetrised hybrid.
  pcg       preconditioned conjugate gradients (Fletcher-Reeves or the flexible
            Polak-Ribiere beta) and the Lanczos estimate of the condition number.
  projection  initial guesses by projection onto prior solutions (Sec. 5).
  problem   glue: one call from a mesh to an assembled preconditioner and solve.

Pins: see tests/test_oracle_*.py. Parity unpinned: the iteration counts on the
synthetic workloads (the paper prints none for them); they are compared between
oracle and GPU only.
"""
from . import fem, schwarz, reduced, precond, pcg, problem  # noqa: F401
