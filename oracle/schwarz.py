"""Overlapping Schwarz local part — oracle (test infrastructure).

Sec. 3: each subdomain Omega_p (a set of elements) is extended by layers of
neighbouring elements into the overlapping subdomain bar-Omega_p; R_p picks the
nodal values interior to bar-Omega_p (those not on its boundary); the local
systems are the principal submatrices A_p = R_p A R_p^T and the local part of
eq. (asm) is sum_p R_p^T A_p^{-1} R_p r (classic ASM, tilde-R_p = R_p).

Readings: one "layer" adds every element sharing at least one vertex with the
current set; a vertex is interior to bar-Omega_p when every element containing it
belongs to bar-Omega_p (so vertices on the physical Neumann boundary stay,
vertices on the artificial boundary go), and Dirichlet vertices never appear.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def vertex_element_incidence(e2v, n_vert):
    """Sparse Boolean (n_vert x n_elem) incidence: vertex u lies in element e."""
    e2v = np.asarray(e2v, dtype=np.int64)
    E = e2v.shape[0]
    rows = e2v.ravel()
    cols = np.repeat(np.arange(E), 8)
    return sp.csr_matrix((np.ones(rows.size, dtype=np.int8), (rows, cols)), shape=(n_vert, E))


def overlapping_subdomains(e2v, part, n_part, layers=1):
    """bar-Omega_p for every p: the elements of Omega_p plus ``layers`` rings of
    elements that share a vertex with the set built so far."""
    e2v = np.asarray(e2v, dtype=np.int64)
    inc = vertex_element_incidence(e2v, int(e2v.max()) + 1)
    part = np.asarray(part)
    order = np.argsort(part, kind="stable")
    bounds = np.searchsorted(part[order], np.arange(n_part + 1))
    out = []
    for p in range(n_part):
        elems = order[bounds[p]:bounds[p + 1]]
        for _ in range(layers):
            verts = np.unique(e2v[elems].ravel())
            elems = np.unique(inc[verts].indices)
        out.append(elems)
    return out


def restriction_sets(e2v, elem_sets, dirichlet):
    """R_p as sorted arrays of (user) vertex ids: free vertices of bar-Omega_p all
    of whose elements lie in bar-Omega_p."""
    e2v = np.asarray(e2v, dtype=np.int64)
    n_vert = len(dirichlet)
    mult = np.bincount(e2v.ravel(), minlength=n_vert)
    dirichlet = np.asarray(dirichlet).astype(bool)
    sets = []
    for elems in elem_sets:
        verts, counts = np.unique(e2v[elems].ravel(), return_counts=True)
        keep = (counts == mult[verts]) & ~dirichlet[verts]
        sets.append(verts[keep])
    return sets


class LocalSolves:
    """Exact local solves A_p^{-1} by dense Cholesky of the principal submatrices
    of A (in free numbering), applied additively: z = sum_p R_p^T A_p^{-1} R_p r."""

    def __init__(self, A, R_free):
        self.R = [np.asarray(R, dtype=np.int64) for R in R_free]
        self.n = A.shape[0]
        A = A.tocsr()
        self.factors = []
        for R in self.R:
            Ap = A[R][:, R].toarray()
            self.factors.append(sla.cho_factor(Ap, lower=True))

    def apply(self, r):
        z = np.zeros(self.n)
        for R, cf in zip(self.R, self.factors):
            z[R] += sla.cho_solve(cf, r[R])
        return z

    def apply_one(self, p, r):
        """A_p^{-1} R_p r for a single subdomain (used for sampled checks)."""
        return sla.cho_solve(self.factors[p], r[self.R[p]])


def local_solves_for(A, R_free, which):
    """Factor only the subdomains listed in ``which`` (sampled checks at sizes
    where factoring every subdomain would take too long)."""
    A = A.tocsr()
    return {p: sla.cho_factor(A[R_free[p]][:, R_free[p]].toarray(), lower=True) for p in which}


def local_part_at(A, R_free, rows, r):
    """Entries ``rows`` (free numbering) of the local part sum_p R_p^T A_p^{-1} R_p r,
    computed from only the subdomains whose R_p contains one of those rows. Each
    entry is the full sum over every subdomain covering it, so it equals the
    corresponding entry of :meth:`LocalSolves.apply` on the whole mesh."""
    rows = np.asarray(rows, dtype=np.int64)
    which = [p for p, R in enumerate(R_free) if np.isin(rows, R, assume_unique=False).any()]
    factors = local_solves_for(A, R_free, which)
    out = np.zeros(rows.size)
    for p in which:
        R = np.asarray(R_free[p], dtype=np.int64)
        zp = sla.cho_solve(factors[p], r[R])
        order = np.argsort(R, kind="stable")
        pos = np.minimum(np.searchsorted(R[order], rows), R.size - 1)
        hit = R[order][pos] == rows
        out[hit] += zp[order[pos[hit]]]
    return out, which


class InexactLocalSolves:
    """Inexact local solves: on every subdomain, k iterations of conjugate
    gradients preconditioned by the diagonal of A_p (Jacobi), from a zero initial
    guess, in place of A_p^{-1} (the paper's suggestion, in its conclusions, of an
    iterative method such as preconditioned CG as an inexact local solver on the
    GPU). The local corrections are summed as in eq. (asm). The result depends
    on r nonlinearly (the CG coefficients are formed from it), so an outer Krylov
    method must be the flexible one."""

    def __init__(self, A, R_free, iters):
        self.R = [np.asarray(R, dtype=np.int64) for R in R_free]
        self.n = A.shape[0]
        self.k = int(iters)
        A = A.tocsr()
        self.A_p = [A[R][:, R].tocsr() for R in self.R]
        self.dinv = [1.0 / Ap.diagonal() for Ap in self.A_p]

    @staticmethod
    def jacobi_pcg(Ap, dinv, b, k):
        """k steps of Jacobi-preconditioned CG on Ap x = b from x = 0."""
        x = np.zeros_like(b)
        r = b.copy()
        z = dinv * r
        p = z.copy()
        rz = float(r @ z)
        for it in range(k):
            if rz == 0.0:
                break
            q = Ap @ p
            alpha = rz / float(p @ q)
            x += alpha * p
            r -= alpha * q
            if it == k - 1:
                break
            z = dinv * r
            rz_new = float(r @ z)
            p = z + (rz_new / rz) * p
            rz = rz_new
        return x

    def apply(self, r):
        z = np.zeros(self.n)
        for R, Ap, dinv in zip(self.R, self.A_p, self.dinv):
            z[R] += self.jacobi_pcg(Ap, dinv, r[R], self.k)
        return z
