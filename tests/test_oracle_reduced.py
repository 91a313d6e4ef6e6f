"""Pins for the oracle's reduced coarse space (Sec. 4): special cases with a
closed-form answer, the exactness of trilinear interpolation on linear fields,
the stencil and size counts the paper prints, and an independent sparse
triple-product construction of the cell-assembled A_r."""
import json
import os

import numpy as np
import scipy.sparse as sp

from oracle import fem, reduced
from paper_2606_20496_amd import meshgen as mg

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")))
GOLD = {it["id"]: it for it in GOLD["items"]}


def _space(m):
    A, Ae, Afull, free, fidx = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
    mult = fem.multiplicity(m.e2v, m.n_vert)
    return A, reduced.CentroidSpace(m.xyz, m.e2v, m.dirichlet, Ae, m.boxes, fidx, mult), free


def test_one_box_per_element_is_identity():
    # Unjittered cube, b = n: each element is a cell, its vertices are the cell
    # corners, so J = I on the free vertices, A_r = A and J A_r^{-1} J^T = A^{-1}.
    n = 4
    m = mg.box_mesh(n, 0, block=2, boxes=(n, n, n), jitter=0.0, permute=True)
    A, S, free = _space(m)
    assert S.n_r == A.shape[0]
    Jd = S.J.toarray()
    # J is a permutation matrix (box-vertex numbering differs from user numbering)
    assert np.allclose(np.sort(Jd, axis=1)[:, -1], 1.0) and np.abs(Jd).sum() == A.shape[0]
    P = Jd
    assert np.abs(P.T @ A.toarray() @ P - S.Ar).max() < 1e-14
    r = np.random.default_rng(0).standard_normal(A.shape[0])
    assert np.abs(S.apply(r) - np.linalg.solve(A.toarray(), r)).max() < 1e-12 * np.abs(S.apply(r)).max()


def test_linear_fields_reproduced():
    # Trilinear interpolation (with extrapolation outside the cell) reproduces any
    # linear function, and averaging equal values changes nothing.
    for m in (mg.box_mesh(9, 2, block=3, boxes=(2, 3, 4), jitter=0.2),
              mg.annulus_mesh(8, 3, block=4, boxes=(3, 3, 2))):
        A, S, free = _space(m)
        nx1, ny1 = S.b[0] + 1, S.b[1] + 1
        ids = S.active
        gi = np.stack([ids % nx1, (ids // nx1) % ny1, ids // (nx1 * ny1)], 1)
        pos = S.lo + gi * S.H
        a = np.array([0.7, -1.3, 2.1])
        y = pos @ a + 0.5
        want = m.xyz[free] @ a + 0.5
        assert np.abs(S.J @ y - want).max() < 1e-13


def test_box_vertex_counts():
    m = mg.box_mesh(8, 1, block=4, boxes=(2, 2, 2))
    _, S, _ = _space(m)
    assert S.n_r == 27
    m = mg.annulus_mesh(16, 3, block=8, boxes=(4, 4, 4))
    _, S, _ = _space(m)
    assert S.n_r < 125            # corners of boxes outside the annulus are dropped
    assert S.n_r > 0


def test_paper_nominal_reduced_dofs():
    g = GOLD["pebble146_nominal_dofs"]
    bx, by, bz = g["boxes"]
    m = mg.box_mesh((2 * bx, 2 * by, 2 * bz), 4, block=4, boxes=(bx, by, bz))
    _, S, _ = _space(m)
    assert S.n_r == g["n_r"]


def test_compact_stencil_width():
    g = GOLD["Ar_row_nnz_compact"]["value"]
    m = mg.box_mesh(12, 5, block=4, boxes=(4, 4, 4), jitter=0.2)
    _, S, _ = _space(m)
    nnz = np.diff(S.Ar_sparse.indptr)
    nz_actual = np.array([np.count_nonzero(S.Ar[i]) for i in range(S.n_r)])
    assert nz_actual.max() == g
    # interior box vertices (not on the bounding box) have the full 3^3 stencil
    ids = S.active
    nx1, ny1 = S.b[0] + 1, S.b[1] + 1
    gi = np.stack([ids % nx1, (ids // nx1) % ny1, ids // (nx1 * ny1)], 1)
    inner = np.all((gi > 0) & (gi < S.b), axis=1)
    assert np.all(nz_actual[inner] == g) and nnz.max() <= g


def test_cell_assembly_equals_triple_product():
    # A_r = S^T J_L^T A_L^masked J_L S built as one sparse product (separate path).
    m = mg.box_mesh(7, 8, block=3, boxes=(3, 2, 3), jitter=0.2, faces=("y0",))
    A, Ae, Afull, free, fidx = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
    mult = fem.multiplicity(m.e2v, m.n_vert)
    S = reduced.CentroidSpace(m.xyz, m.e2v, m.dirichlet, Ae, m.boxes, fidx, mult)
    E = m.n_elem
    AL = sp.block_diag([Ae[e] for e in range(E)], format="csr")
    D = sp.diags((~m.dirichlet.astype(bool)[m.e2v]).astype(float).ravel())
    AL = D @ AL @ D                               # Dirichlet rows/columns of A^e removed
    nbv = int(np.prod(S.b + 1))
    corners = reduced.corner_ids(S.cells, S.b)
    Smat = sp.csr_matrix((np.ones(E * 8), (np.arange(E * 8), corners.ravel())), shape=(E * 8, nbv))
    xi = (m.xyz[m.e2v] - S.lo - S.cells[:, None, :] * S.H) / S.H
    JL = sp.block_diag([reduced.trilinear_weights(xi[e]) for e in range(E)], format="csr")
    Ar = (Smat.T @ JL.T @ AL @ JL @ Smat).toarray()[np.ix_(S.active, S.active)]
    assert np.abs(Ar - S.Ar).max() < 1e-13 * np.abs(Ar).max()


def test_aligned_boxes_match_galerkin():
    # Unjittered mesh whose element faces lie on the cell planes: every element
    # lies in one cell, J^e equals the rows of the continuous J, so the
    # cell-assembled A_r is exactly the Galerkin J^T A J of the standard space.
    m = mg.box_mesh(8, 9, block=4, boxes=(2, 4, 2), jitter=0.0, faces=("x1",))
    A, Ae, Afull, free, fidx = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
    mult = fem.multiplicity(m.e2v, m.n_vert)
    C = reduced.CentroidSpace(m.xyz, m.e2v, m.dirichlet, Ae, m.boxes, fidx, mult)
    G = reduced.StandardSpace(m.xyz, m.dirichlet, A, m.boxes, free)
    assert np.array_equal(C.active, G.active)
    assert np.abs((C.J - G.J).toarray()).max() < 1e-15
    assert np.abs(C.Ar - G.Ar).max() < 1e-13 * np.abs(G.Ar).max()


def test_standard_space_counts_and_best_approximation():
    m = mg.box_mesh(16, 6, block=4, boxes=(4, 4, 4), jitter=0.2)
    A, Ae, Afull, free, fidx = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
    G = reduced.StandardSpace(m.xyz, m.dirichlet, A, m.boxes, free)
    row_nnz = np.diff(G.J.indptr)
    assert row_nnz.max() == GOLD["J_row_nnz"]["value"]
    nz = np.array([np.count_nonzero(np.abs(G.Ar[i]) > 1e-14 * np.abs(G.Ar).max()) for i in range(G.n_r)])
    ids = G.active
    nx1, ny1 = G.b[0] + 1, G.b[1] + 1
    gi = np.stack([ids % nx1, (ids // nx1) % ny1, ids // (nx1 * ny1)], 1)
    inner = np.all((gi >= 2) & (gi <= G.b - 2), axis=1)
    # at most 5^3 couplings per row, and well beyond the compact 3^3 in the interior
    # (which of the 125 appear depends on which elements straddle cell planes)
    assert nz.max() <= GOLD["Ar_row_nnz_standard"]["value"]
    assert inner.any() and np.all(nz[inner] > GOLD["Ar_row_nnz_compact"]["value"] * 4)
    # Galerkin: z_r = J A_r^{-1} J^T r is the A-orthogonal projection of A^{-1} r,
    # so the residual r - A z_r is orthogonal to range(J).
    r = np.random.default_rng(3).standard_normal(A.shape[0])
    zr = G.apply(r)
    assert np.abs(G.J.T @ (r - A @ zr)).max() < 1e-11 * np.abs(G.J.T @ r).max()


def test_one_dimensional_stencils():
    # 1D analogue (Fig. of 1D reduced bases): a thin bar of elements, one box across
    # y and z, many along x. Standard support couples box vertices two apart
    # (width 5); the centroid scheme only neighbours (width 3).
    g = GOLD["stencil_1d"]
    m = mg.box_mesh((24, 2, 2), 7, block=24, boxes=(6, 1, 1), jitter=0.3, faces=("x0",))
    A, Ae, Afull, free, fidx = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
    mult = fem.multiplicity(m.e2v, m.n_vert)
    C = reduced.CentroidSpace(m.xyz, m.e2v, m.dirichlet, Ae, m.boxes, fidx, mult)
    G = reduced.StandardSpace(m.xyz, m.dirichlet, A, m.boxes, free)

    def width(S):
        ix = S.active % (S.b[0] + 1)
        w = 0
        for i in range(S.n_r):
            cols = np.flatnonzero(np.abs(S.Ar[i]) > 1e-14 * np.abs(S.Ar).max())
            w = max(w, 2 * int(np.abs(ix[cols] - ix[i]).max()) + 1)
        return w
    # with jitter, elements straddle the cell planes: the standard space sees them
    assert width(G) == g["standard"]
    assert width(C) == g["compact"]


def test_reduced_operator_spd():
    m = mg.annulus_mesh(12, 1, block=4, boxes=(3, 3, 3))
    _, S, _ = _space(m)
    assert np.abs(S.Ar - S.Ar.T).max() < 1e-13 * np.abs(S.Ar).max()
    assert np.linalg.eigvalsh(S.Ar)[0] > 0
