"""Q1 (trilinear, N=1) finite-element Poisson operator — oracle (test infrastructure).

Sec. 3: A = Q^T A_L Q with A_L = block-diag(A^e) and
a^e_ij = integral over element e of grad l_i . grad l_j.
Each hexahedron is the trilinear (isoparametric) image of the reference cube
[-1,1]^3 (Sec. 1); the integral uses the tensor 2x2x2 Gauss-Legendre rule
(points +-1/sqrt(3), unit weights), which is the "suitable quadrature" reading.
Local vertex v = i + 2j + 4k sits at reference point (2i-1, 2j-1, 2k-1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_G = 1.0 / np.sqrt(3.0)
GAUSS_POINTS = [(a, b, c) for c in (-_G, _G) for b in (-_G, _G) for a in (-_G, _G)]
REF_VERTS = np.array([[2 * (v & 1) - 1, 2 * ((v >> 1) & 1) - 1, 2 * ((v >> 2) & 1) - 1]
                      for v in range(8)], dtype=np.float64)


def ref_gradients(xi):
    """Gradients (8, 3) of the trilinear reference basis N_v at point xi in [-1,1]^3:
    N_v = prod_d (1 + s_vd xi_d) / 8 with s_v the vertex signs."""
    xi = np.asarray(xi, dtype=np.float64)
    s = REF_VERTS
    f = 1.0 + s * xi[None, :]          # (8, 3)
    g = np.empty((8, 3))
    g[:, 0] = s[:, 0] * f[:, 1] * f[:, 2] / 8.0
    g[:, 1] = s[:, 1] * f[:, 0] * f[:, 2] / 8.0
    g[:, 2] = s[:, 2] * f[:, 0] * f[:, 1] / 8.0
    return g


def element_matrices(xyz, e2v):
    """A^e for every element (E, 8, 8) and the minimum Jacobian determinant over
    the quadrature points of each element (E,).

    A^e_ij = sum_q w_q |J_q| (J_q^{-T} gN_i) . (J_q^{-T} gN_j), J_q = dx/dxi."""
    X = np.asarray(xyz, dtype=np.float64)[np.asarray(e2v)]      # (E, 8, 3)
    E = X.shape[0]
    A = np.zeros((E, 8, 8))
    detmin = np.full(E, np.inf)
    for q in GAUSS_POINTS:
        gN = ref_gradients(q)                                   # (8, 3)
        Jac = np.matmul(X.transpose(0, 2, 1), gN)              # J_ij = dx_i/dxi_j
        det = np.linalg.det(Jac)
        detmin = np.minimum(detmin, det)
        inv = np.linalg.inv(Jac)                                # (E, 3, 3)
        G = np.matmul(gN[None, :, :], inv)                      # physical gradients (E, 8, 3)
        A += det[:, None, None] * np.matmul(G, G.transpose(0, 2, 1))
    return A, detmin


def element_magnitudes(xyz, e2v, conditioned=False):
    """The same sum as :func:`element_matrices` taken in absolute values,
    sum_q |J_q| |G_q| |G_q|^T (E, 8, 8): the magnitude that bounds the rounding
    error of the products with A^e. With ``conditioned`` each quadrature term is
    weighted by the 2-norm condition number of J_q, since the physical gradients
    G_q = gN J_q^{-1} carry a relative rounding error of order cond(J_q) eps."""
    X = np.asarray(xyz, dtype=np.float64)[np.asarray(e2v)]
    M = np.zeros((X.shape[0], 8, 8))
    for q in GAUSS_POINTS:
        gN = ref_gradients(q)
        Jac = np.matmul(X.transpose(0, 2, 1), gN)
        G = np.abs(np.matmul(gN[None, :, :], np.linalg.inv(Jac)))
        w = np.abs(np.linalg.det(Jac))
        if conditioned:
            w = w * np.linalg.cond(Jac)
        M += w[:, None, None] * np.matmul(G, G.transpose(0, 2, 1))
    return M


def assemble(Ae, e2v, n_vert):
    """A_full = Q^T A_L Q as a sparse (n_vert x n_vert) matrix: the local-to-global
    summation of Sec. 3 (duplicates summed)."""
    e2v = np.asarray(e2v, dtype=np.int64)
    rows = np.repeat(e2v, 8, axis=1).ravel()
    cols = np.tile(e2v, (1, 8)).ravel()
    return sp.coo_matrix((Ae.reshape(-1), (rows, cols)), shape=(n_vert, n_vert)).tocsr()


def multiplicity(e2v, n_vert):
    """Counting vector w = Q Q^T e_L: number of elements sharing each vertex (Sec. 4)."""
    return np.bincount(np.asarray(e2v).ravel(), minlength=n_vert).astype(np.int64)


def free_numbering(dirichlet):
    """Free (non-Dirichlet) vertices in increasing user order, and the map
    vertex -> free index (-1 for Dirichlet). Basis functions vanish on the
    Dirichlet boundary (Sec. 3), so those rows and columns are removed."""
    dirichlet = np.asarray(dirichlet).astype(bool)
    free = np.flatnonzero(~dirichlet)
    fidx = np.full(dirichlet.size, -1, dtype=np.int64)
    fidx[free] = np.arange(free.size)
    return free, fidx


def stiffness(xyz, e2v, dirichlet):
    """The coarse system matrix A (free rows and columns) plus pieces reused by
    the preconditioner: element matrices, the full assembled matrix and the free
    numbering."""
    Ae, detmin = element_matrices(xyz, e2v)
    if np.any(detmin <= 0):
        raise ValueError("element with non-positive Jacobian determinant")
    Afull = assemble(Ae, e2v, len(xyz))
    free, fidx = free_numbering(dirichlet)
    A = Afull[free][:, free].tocsr()
    return A, Ae, Afull, free, fidx
