"""Initial guess by projection onto prior solutions — oracle (test infrastructure).

Sec. 5: for a sequence of right-hand sides with the same matrix, the solver works
on the change from the A-orthogonal (best fit) projection of the new solution onto
the span of l prior solutions. The basis x_1 .. x_l is kept A-orthonormal
(x_j^T A x_k = delta_jk) together with A x_j, so that for a new b

    c_j = x_j^T b,   u_bar = sum_j c_j x_j,   r_0 = b - sum_j c_j (A x_j)

(u_bar minimises the A-norm error over the span), PCG solves A d = r_0 to the
tolerance relative to ||b||, and u = u_bar + d. Then u joins the basis by
A-Gram-Schmidt: with A u, e_j = x_j^T (A u), w = u - sum_j e_j x_j,
A w = A u - sum_j e_j (A x_j), w and A w scaled by 1/sqrt(w^T A w); a w whose
A-norm is below 1e-6 of that of u is dropped (u is already in the span). When the
basis is full it restarts from the new solution alone. Vectors are free-vertex
vectors.
"""
from __future__ import annotations

import numpy as np

from . import pcg as _pcg


class Projection:
    def __init__(self, max_vectors):
        self.L = int(max_vectors)
        self.X, self.AX = [], []

    def initial_guess(self, b):
        """(u_bar, r_0) for right-hand side b."""
        u = np.zeros_like(b)
        r = b.copy()
        for x, ax in zip(self.X, self.AX):
            c = float(x @ b)
            u += c * x
            r -= c * ax
        return u, r

    def add(self, u, Au):
        """A-orthonormalise u against the basis and append it (restart when full)."""
        if len(self.X) >= self.L:
            self.X, self.AX = [], []
        w, aw = u.copy(), Au.copy()
        for x, ax in zip(self.X, self.AX):
            e = float(x @ Au)
            w -= e * x
            aw -= e * ax
        nrm2 = float(w @ aw)
        # a solution already in the span (to 1e-6 in the A-norm) adds only noise
        if nrm2 > 1e-12 * float(u @ Au) and np.isfinite(nrm2):
            s = 1.0 / np.sqrt(nrm2)
            self.X.append(w * s)
            self.AX.append(aw * s)


def solve_projected(matvec, precond, b, proj, tol=1e-8, max_it=1000, flexible=False):
    """One solve of the sequence: projection, PCG on the remainder (stopping at
    ||r|| <= tol ||b||), basis update. Returns (u, info) with info["iters"] the PCG
    iterations after the projection."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.sqrt(b @ b))
    ubar, r0 = proj.initial_guess(b)
    r0norm = float(np.sqrt(r0 @ r0))
    if bnorm == 0.0 or r0norm <= tol * bnorm:
        d, info = np.zeros_like(b), {"iters": 0, "relres": r0norm / bnorm if bnorm else 0.0}
    else:
        d, info = _pcg.pcg(matvec, precond, r0, tol=tol * bnorm / r0norm, max_it=max_it, flexible=flexible)
    u = ubar + d
    proj.add(u, matvec(u))
    info = dict(info)
    info["r0_rel"] = r0norm / bnorm if bnorm else 0.0
    return u, info
