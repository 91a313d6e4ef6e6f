"""Two-level Schwarz preconditioners — oracle (test infrastructure).

Sec. 3, eq. (asm): z = sum_p R_p^T A_p^{-1} R_p r + J A_r^{-1} J^T r.
Also the hybrid forms of eqs. (asm1)-(asm2). The paper's hybrid (local step, then
a coarse correction of the updated residual) is not symmetric, so for use under
CG this module offers the symmetrised coarse-local-coarse sweep
  z0 = M_r r,  z1 = z0 + M_loc (r - A z0),  z = z1 + M_r (r - A z1),
with M_r = J A_r^{-1} J^T and M_loc = sum_p R_p^T A_p^{-1} R_p; and the paper's
two-step form ASM_1 -> ASM_2 as written (for flexible Krylov methods).
"""
from __future__ import annotations


class Additive:
    """eq. (asm)."""

    def __init__(self, local, coarse):
        self.local, self.coarse = local, coarse

    def __call__(self, r):
        return self.local.apply(r) + self.coarse.apply(r)


class LocalOnly:
    """eq. (asm1) alone (the paper's 'ASM_1 only' ablation)."""

    def __init__(self, local):
        self.local = local

    def __call__(self, r):
        return self.local.apply(r)


class CoarseOnly:
    """M_r alone (the paper's 'reduced-space solver only' ablation)."""

    def __init__(self, coarse):
        self.coarse = coarse

    def __call__(self, r):
        return self.coarse.apply(r)


class HybridPaper:
    """eqs. (asm1)-(asm2): z_loc = M_loc r; z = z_loc + M_r (r - A z_loc)."""

    def __init__(self, A, local, coarse):
        self.A, self.local, self.coarse = A, local, coarse

    def __call__(self, r):
        zl = self.local.apply(r)
        return zl + self.coarse.apply(r - self.A @ zl)


class HybridSymmetric:
    """Coarse-local-coarse symmetrised hybrid (symmetric whenever M_loc is)."""

    def __init__(self, A, local, coarse):
        self.A, self.local, self.coarse = A, local, coarse

    def __call__(self, r):
        z0 = self.coarse.apply(r)
        z1 = z0 + self.local.apply(r - self.A @ z0)
        return z1 + self.coarse.apply(r - self.A @ z1)
