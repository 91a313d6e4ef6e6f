"""Non-nested reduced coarse space on a box grid — oracle (test infrastructure).

Sec. 4. The bounding box of the domain is cut into b_x x b_y x b_z boxes; the
reduced basis functions Phi_j are the trilinear interpolants attached to the box
vertices, lexicographically ordered (Sec. 4, construction of J). Two variants:

* ``centroid`` (the default, used by the paper's experiments): every element is
  assigned to the cell containing its centroid and uses that cell's trilinear
  interpolant J^e (n_v x 2^d) for all its vertices; the discontinuous result is
  made continuous by W Q^T (W = diag(1/w), w = Q Q^T e_L the counting vector).
  So J = W Q^T J_L S, and A_r is built by cell assembly, eq. (Aij):
  A_r = sum_e S_e^T (J^e)^T A^e J^e S_e (a 3^d-point stencil).
* ``standard``: J_ij = Phi_j(x_i) using the box that bounds node x_i (2^d nonzeros
  per row), with the Galerkin reduced operator A_r = J^T A J (a 5^d stencil).

Readings: the bounding box is the min/max of all vertex coordinates and
H = (hi - lo)/b; the element centroid is the plain mean of its 8 vertices,
summed in local vertex order; the cell index is floor((c - lo)/H) clamped to
[0, b-1]; local coordinates xi = ((x - lo) - c H)/H may leave [0,1]
(extrapolation); rows of J at Dirichlet vertices are zero (the Psi_j inherit the
boundary conditions); box vertices whose column of J has no nonzero entry are
compressed out; the restriction is the exact transpose of J, which keeps the
preconditioner symmetric.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def bounding_box(xyz, boxes):
    """lo, hi and box size H of the reduced grid (Sec. 4: limits of Omega in each
    principal direction, split into b_x x b_y x b_z boxes)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    lo = xyz.min(axis=0)
    hi = xyz.max(axis=0)
    b = np.asarray(boxes, dtype=np.int64)
    H = (hi - lo) / b
    return lo, hi, H, b


def element_centroids(xyz, e2v):
    """Mean of the 8 vertex coordinates of each element, summed in local order."""
    X = np.asarray(xyz, dtype=np.float64)[np.asarray(e2v)]
    s = X[:, 0, :].copy()
    for v in range(1, 8):
        s = s + X[:, v, :]
    return s / 8.0


def cell_of_points(pts, lo, H, b):
    """Integer cell (box) coordinates of points: floor((x - lo)/H) clamped."""
    c = np.floor((pts - lo) / H).astype(np.int64)
    return np.clip(c, 0, b - 1)


def local_coords(x, cells, lo, H):
    """xi = ((x - lo) - c H) / H, per coordinate."""
    return ((x - lo) - cells * H) / H


def trilinear_weights(xi):
    """Phi_k at local coordinates xi (..., 3) for the 8 corners k = kx + 2ky + 4kz:
    product over d of (xi_d if k_d == 1 else 1 - xi_d)."""
    xi = np.asarray(xi)
    out = np.empty(xi.shape[:-1] + (8,))
    for k in range(8):
        kx, ky, kz = k & 1, (k >> 1) & 1, (k >> 2) & 1
        fx = xi[..., 0] if kx else 1.0 - xi[..., 0]
        fy = xi[..., 1] if ky else 1.0 - xi[..., 1]
        fz = xi[..., 2] if kz else 1.0 - xi[..., 2]
        out[..., k] = fx * fy * fz
    return out


def corner_ids(cells, b):
    """Lexicographic ids of the 8 box vertices (corners) of each cell."""
    nx1, ny1 = b[0] + 1, b[1] + 1
    ids = np.empty(cells.shape[:-1] + (8,), dtype=np.int64)
    for k in range(8):
        kx, ky, kz = k & 1, (k >> 1) & 1, (k >> 2) & 1
        ids[..., k] = (cells[..., 0] + kx) + nx1 * ((cells[..., 1] + ky) + ny1 * (cells[..., 2] + kz))
    return ids


class CentroidSpace:
    """Element-centroid reduced space: J (n_free x n_r, sparse), A_r (dense) and
    its Cholesky factor."""

    def __init__(self, xyz, e2v, dirichlet, Ae, boxes, free_index, mult):
        xyz = np.asarray(xyz, dtype=np.float64)
        e2v = np.asarray(e2v, dtype=np.int64)
        self.lo, self.hi, self.H, self.b = bounding_box(xyz, boxes)
        nbv = int(np.prod(self.b + 1))
        self.cells = cell_of_points(element_centroids(xyz, e2v), self.lo, self.H, self.b)
        corners = corner_ids(self.cells, self.b)                       # (E, 8)
        xi = local_coords(xyz[e2v], self.cells[:, None, :], self.lo, self.H)   # (E, 8, 3)
        Je = trilinear_weights(xi)                                      # (E, 8 verts, 8 corners)
        dmask = np.asarray(dirichlet).astype(bool)[e2v]                 # (E, 8)
        Je[dmask] = 0.0
        self.Je = Je
        # J = W Q^T J_L S on free rows
        rows = np.repeat(free_index[e2v], 8, axis=1).reshape(-1)        # vertex of (e, a), repeated per k
        cols = np.tile(corners, (1, 8)).reshape(-1)
        w = 1.0 / mult[e2v]                                            # (E, 8)
        vals = (Je * w[:, :, None]).reshape(-1)
        keep = rows >= 0
        n_free = int(free_index.max()) + 1
        Jfull = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n_free, nbv)).tocsc()
        Jfull.sum_duplicates()
        colnz = np.diff(Jfull.indptr) > 0
        nzcount = np.zeros(nbv, dtype=bool)
        for j in np.flatnonzero(colnz):
            seg = Jfull.data[Jfull.indptr[j]:Jfull.indptr[j + 1]]
            nzcount[j] = bool(np.any(seg != 0.0))
        self.active = np.flatnonzero(nzcount)                          # compressed box vertices
        self.n_r = self.active.size
        self.J = Jfull[:, self.active].tocsr()
        # A_r by cell assembly, eq. (Aij): sum_e (J^e)^T A^e J^e at the cell corners
        Acell = np.matmul(np.matmul(Je.transpose(0, 2, 1), Ae), Je)   # (J^e)^T A^e J^e
        r_ = np.repeat(corners, 8, axis=1).reshape(-1)
        c_ = np.tile(corners, (1, 8)).reshape(-1)
        Arfull = sp.coo_matrix((Acell.reshape(-1), (r_, c_)), shape=(nbv, nbv)).tocsr()
        self.Ar_sparse = Arfull[self.active][:, self.active].tocsr()
        self.Ar = self.Ar_sparse.toarray()
        self.factor = sla.cho_factor(self.Ar, lower=True)

    def restrict(self, r):
        return self.J.T @ r

    def solve_reduced(self, rr):
        return sla.cho_solve(self.factor, rr)

    def prolong(self, y):
        return self.J @ y

    def apply(self, r):
        """J A_r^{-1} J^T r (the reduced term of eq. (asm))."""
        return self.prolong(self.solve_reduced(self.restrict(r)))


class StandardSpace:
    """Vertex-based reduced space: J_ij = Phi_j(x_i) with the box that bounds x_i,
    A_r = J^T A J (Galerkin, Sec. 4 eq. (Psi) and the reduced system)."""

    def __init__(self, xyz, dirichlet, A, boxes, free):
        xyz = np.asarray(xyz, dtype=np.float64)
        self.lo, self.hi, self.H, self.b = bounding_box(xyz, boxes)
        nbv = int(np.prod(self.b + 1))
        pts = xyz[free]
        cells = cell_of_points(pts, self.lo, self.H, self.b)
        w = trilinear_weights(local_coords(pts, cells, self.lo, self.H))
        ids = corner_ids(cells, self.b)
        rows = np.repeat(np.arange(free.size), 8)
        Jfull = sp.coo_matrix((w.reshape(-1), (rows, ids.reshape(-1))), shape=(free.size, nbv)).tocsc()
        Jfull.sum_duplicates()
        nz = np.zeros(nbv, dtype=bool)
        for j in range(nbv):
            seg = Jfull.data[Jfull.indptr[j]:Jfull.indptr[j + 1]]
            nz[j] = bool(np.any(seg != 0.0))
        self.active = np.flatnonzero(nz)
        self.n_r = self.active.size
        self.J = Jfull[:, self.active].tocsr()
        self.Ar_sparse = (self.J.T @ A @ self.J).tocsr()
        self.Ar = self.Ar_sparse.toarray()
        self.factor = sla.cho_factor(self.Ar, lower=True)

    def apply(self, r):
        return self.J @ sla.cho_solve(self.factor, self.J.T @ r)
