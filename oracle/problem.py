"""Glue from a mesh to the oracle's operator, preconditioner and solve — oracle
(test infrastructure).

Vectors at this level have one entry per mesh vertex in the caller's numbering
(Dirichlet entries ignored on input, zero on output), the same convention as the
GPU library's boundary; internally everything works on the free vertices.
"""
from __future__ import annotations

import numpy as np

from . import fem, schwarz, reduced, precond, pcg


class Problem:
    """Sec. 3-4 assembled once per mesh.

    interp: "centroid" (cell-assembled A_r, default) or "standard" (Galerkin).
    local_iters: 0 (exact local solves) or k > 0 (k steps of Jacobi-PCG per
            subdomain; nonlinear in r, so solve with ``flexible=True``).
    mode:   "additive" (eq. (asm)), "hybrid" (eqs. (asm1)-(asm2) as written; not
            symmetric, so solve with ``flexible=True``), "hybrid_sym",
            "local_only", "coarse_only".
    """

    def __init__(self, xyz, e2v, dirichlet, part, n_part, boxes, overlap=1,
                 interp="centroid", mode="additive", local_iters=0):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.e2v = np.asarray(e2v, dtype=np.int64)
        self.dirichlet = np.asarray(dirichlet).astype(bool)
        self.n_vert = self.xyz.shape[0]
        self.A, self.Ae, self.Afull, self.free, self.fidx = fem.stiffness(self.xyz, self.e2v, self.dirichlet)
        self.mult = fem.multiplicity(self.e2v, self.n_vert)
        self.elem_sets = schwarz.overlapping_subdomains(self.e2v, part, n_part, overlap)
        self.R_user = schwarz.restriction_sets(self.e2v, self.elem_sets, self.dirichlet)
        self.R = [self.fidx[R] for R in self.R_user]
        # exact local solves, or with local_iters = k > 0 k steps of Jacobi-PCG
        self.local = (schwarz.InexactLocalSolves(self.A, self.R, local_iters) if local_iters > 0
                      else schwarz.LocalSolves(self.A, self.R))
        if interp == "centroid":
            self.coarse = reduced.CentroidSpace(self.xyz, self.e2v, self.dirichlet, self.Ae, boxes,
                                                self.fidx, self.mult)
        elif interp == "standard":
            self.coarse = reduced.StandardSpace(self.xyz, self.dirichlet, self.A, boxes, self.free)
        else:
            raise ValueError(interp)
        self.mode = mode
        self.M = {
            "additive": lambda: precond.Additive(self.local, self.coarse),
            "hybrid": lambda: precond.HybridPaper(self.A, self.local, self.coarse),
            "hybrid_sym": lambda: precond.HybridSymmetric(self.A, self.local, self.coarse),
            "local_only": lambda: precond.LocalOnly(self.local),
            "coarse_only": lambda: precond.CoarseOnly(self.coarse),
        }[mode]()

    # free <-> full vectors
    def to_free(self, v):
        return np.asarray(v, dtype=np.float64)[self.free]

    def to_full(self, vf):
        out = np.zeros(self.n_vert)
        out[self.free] = vf
        return out

    def apply_precond(self, r_full):
        return self.to_full(self.M(self.to_free(r_full)))

    def apply_A(self, p_full):
        return self.to_full(self.A @ self.to_free(p_full))

    def solve(self, b_full, tol=1e-8, max_it=1000, flexible=False, record=False):
        bf = self.to_free(b_full)
        x, info = pcg.pcg(lambda v: self.A @ v, self.M, bf, tol=tol, max_it=max_it,
                          flexible=flexible, record=record)
        bn = np.linalg.norm(bf)
        info["relres_true"] = float(np.linalg.norm(bf - self.A @ x) / bn) if bn > 0 else 0.0
        return self.to_full(x), info


def from_mesh(mesh, **kw):
    """Build a :class:`Problem` from any object carrying the generator's fields
    (xyz, e2v, dirichlet, part, n_part, boxes)."""
    return Problem(mesh.xyz, mesh.e2v, mesh.dirichlet, mesh.part, mesh.n_part, mesh.boxes, **kw)
