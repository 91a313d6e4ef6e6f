"""Pins for the oracle's Q1 operator (Sec. 3: a^e_ij = int grad l_i . grad l_j,
A = Q^T A_L Q). Each test checks the oracle against something it does not compute
itself: textbook closed forms, identities of the continuous problem that the
2x2x2 rule reproduces exactly, and brute-force quadrature of the definition."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem
from paper_2606_20496_amd import meshgen as mg


def _box_element(hx, hy, hz, origin=(0.0, 0.0, 0.0)):
    xyz = np.array([[origin[0] + hx * (v & 1), origin[1] + hy * ((v >> 1) & 1),
                     origin[2] + hz * ((v >> 2) & 1)] for v in range(8)])
    return xyz, np.arange(8)[None, :]


def test_unit_cube_closed_form():
    # Textbook Q1 Laplacian on a cube of side h: diagonal h/3, vertices that differ
    # in one coordinate 0, in two coordinates -h/12, in three -h/12.
    for h in (1.0, 0.5, 0.125):
        xyz, e2v = _box_element(h, h, h, origin=(3.0, -1.0, 2.0))
        A, det = fem.element_matrices(xyz, e2v)
        A = A[0]
        for a, b in itertools.product(range(8), range(8)):
            d = bin(a ^ b).count("1")
            want = {0: h / 3, 1: 0.0, 2: -h / 12, 3: -h / 12}[d]
            assert abs(A[a, b] - want) < 1e-15 * max(1.0, h) * 10


def _k1(h):
    return np.array([[1.0, -1.0], [-1.0, 1.0]]) / h


def _m1(h):
    return np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0


def test_box_element_tensor_product():
    # Rectangular box: A^e = Kx(x)My(x)Mz + Mx(x)Ky(x)Mz + Mx(x)My(x)Kz with the 1D
    # stiffness K and mass M (local order v = i + 2j + 4k -> kron order z, y, x).
    hx, hy, hz = 0.3, 0.7, 1.9
    xyz, e2v = _box_element(hx, hy, hz)
    A = fem.element_matrices(xyz, e2v)[0][0]
    want = (np.kron(_m1(hz), np.kron(_m1(hy), _k1(hx)))
            + np.kron(_m1(hz), np.kron(_k1(hy), _m1(hx)))
            + np.kron(_k1(hz), np.kron(_m1(hy), _m1(hx))))
    assert np.abs(A - want).max() < 1e-14


def _assembled_1d(n, h):
    K = sp.lil_matrix((n + 1, n + 1))
    M = sp.lil_matrix((n + 1, n + 1))
    for e in range(n):
        for a in range(2):
            for b in range(2):
                K[e + a, e + b] += _k1(h)[a, b]
                M[e + a, e + b] += _m1(h)[a, b]
    return K.tocsr(), M.tocsr()


def test_unjittered_grid_is_kronecker_sum():
    n = 5
    m = mg.box_mesh(n, 0, block=n, boxes=(1, 1, 1), jitter=0.0, permute=False, faces=())
    A, Ae, Afull, free, fidx = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
    K, M = _assembled_1d(n, 1.0 / n)
    want = sp.kron(M, sp.kron(M, K)) + sp.kron(M, sp.kron(K, M)) + sp.kron(K, sp.kron(M, M))
    assert abs(Afull - want).max() < 1e-14


def _jittered(n=6, seed=11):
    return mg.box_mesh(n, seed, block=3, boxes=(2, 2, 2), jitter=0.2)


def test_symmetry_and_constant_nullspace():
    m = _jittered()
    A, Ae, Afull, free, fidx = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
    assert abs(Afull - Afull.T).max() < 1e-15
    assert np.abs(Afull @ np.ones(m.n_vert)).max() < 1e-14
    # PSD with a one-dimensional null space: eigenvalues of the full matrix
    ev = np.linalg.eigvalsh(Afull.toarray())
    assert ev[0] > -1e-13 and abs(ev[0]) < 1e-13 and ev[1] > 1e-6
    # SPD once the Dirichlet face is removed
    np.linalg.cholesky(A.toarray())


def test_linear_fields_annihilated_at_interior_vertices():
    # sum_j a_ij x_j = int grad phi_i . a = 0 for interior i (divergence theorem);
    # the 2x2x2 rule integrates a . cof(J) grad N exactly on trilinear elements.
    m = _jittered(7, 5)
    _, _, Afull, _, _ = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
    lo, hi = m.xyz.min(0), m.xyz.max(0)
    tol = 1e-12
    on_boundary = np.any(np.isclose(m.xyz, lo, atol=tol) | np.isclose(m.xyz, hi, atol=tol), axis=1)
    for a in (np.array([1.0, 0, 0]), np.array([0.3, -2.0, 0.7])):
        u = m.xyz @ a + 0.25
        res = Afull @ u
        assert np.abs(res[~on_boundary]).max() < 5e-14
        assert np.abs(res[on_boundary]).max() > 1e-3   # boundary rows carry the flux


def test_linear_field_energy_equals_volume():
    # u = a.x has int |grad u|^2 = |a|^2 vol(Omega) = |a|^2 for the unit cube.
    m = _jittered(6, 3)
    _, _, Afull, _, _ = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
    a = np.array([0.4, -1.1, 2.0])
    u = m.xyz @ a
    assert abs(u @ (Afull @ u) - a @ a) < 1e-13 * (a @ a) * 10


def _brute_force_element(X, npts=5):
    # Independent evaluation of the definition with an npts^3 Gauss rule.
    g, w = np.polynomial.legendre.leggauss(npts)
    s = np.array([[2 * (v & 1) - 1, 2 * ((v >> 1) & 1) - 1, 2 * ((v >> 2) & 1) - 1] for v in range(8)])
    A = np.zeros((8, 8))
    for (i, x1), (j, x2), (k, x3) in itertools.product(enumerate(g), repeat=3):
        xi = np.array([x1, x2, x3])
        dN = np.zeros((8, 3))
        for v in range(8):
            f = 1 + s[v] * xi
            dN[v] = [s[v, 0] * f[1] * f[2], s[v, 1] * f[0] * f[2], s[v, 2] * f[0] * f[1]]
        dN /= 8
        Jm = X.T @ dN
        G = dN @ np.linalg.inv(Jm)
        A += w[i] * w[j] * w[k] * np.linalg.det(Jm) * G @ G.T
    return A


def test_affine_element_matches_brute_force():
    # On an affine (parallelepiped) element the 2x2x2 rule is exact.
    rng = np.random.default_rng(0)
    M = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    assert np.linalg.det(M) > 0
    ref = np.array([[v & 1, (v >> 1) & 1, (v >> 2) & 1] for v in range(8)], dtype=float)
    X = ref @ M.T + np.array([0.2, -0.4, 1.0])
    A = fem.element_matrices(X, np.arange(8)[None, :])[0][0]
    assert np.abs(A - _brute_force_element(X)).max() < 1e-13


def test_rigid_motion_and_scaling():
    rng = np.random.default_rng(2)
    X = np.array([[v & 1, (v >> 1) & 1, (v >> 2) & 1] for v in range(8)], float)
    X = X + 0.1 * rng.uniform(-1, 1, X.shape)
    A0 = fem.element_matrices(X, np.arange(8)[None, :])[0][0]
    Qm, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Qm) < 0:
        Qm[:, 0] *= -1
    A1 = fem.element_matrices(X @ Qm.T + 5.0, np.arange(8)[None, :])[0][0]
    A2 = fem.element_matrices(2.5 * X, np.arange(8)[None, :])[0][0]
    assert np.abs(A1 - A0).max() < 1e-13
    assert np.abs(A2 - 2.5 * A0).max() < 1e-13   # 3D stiffness scales like length


def test_inverted_element_rejected():
    xyz, e2v = _box_element(1, 1, 1)
    e2v = e2v[:, [1, 0, 3, 2, 5, 4, 7, 6]]   # mirror in x: negative Jacobian
    with pytest.raises(ValueError):
        fem.stiffness(xyz, e2v, np.zeros(8, np.uint8))


def test_element_magnitudes_bound_the_element_matrices():
    # the absolute-value sum dominates |A^e| entry by entry, equals it on the
    # diagonal (a sum of non-negative terms), and on the unit cube reproduces the
    # closed-form diagonal h/3 of the Q1 stiffness
    m = mg.box_mesh(4, 9, block=2, boxes=(2, 2, 2))
    Ae, _ = fem.element_matrices(m.xyz, m.e2v)
    M = fem.element_magnitudes(m.xyz, m.e2v)
    assert np.all(M >= np.abs(Ae) * (1 - 1e-14))
    d = np.arange(8)
    assert np.allclose(M[:, d, d], Ae[:, d, d], rtol=1e-14, atol=0)
    cube = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)], dtype=float)
    Mc = fem.element_magnitudes(cube, np.arange(8)[None, :])[0]
    assert np.allclose(np.diag(Mc), 1.0 / 3.0, rtol=1e-14)
    # the conditioned form: cond(J) = 1 on the unit cube, = 4 on a 1 x 1 x 1/4 box
    assert np.allclose(fem.element_magnitudes(cube, np.arange(8)[None, :], conditioned=True)[0], Mc, rtol=1e-14)
    flat = cube * np.array([1.0, 1.0, 0.25])
    assert np.allclose(fem.element_magnitudes(flat, np.arange(8)[None, :], conditioned=True)[0],
                       4.0 * fem.element_magnitudes(flat, np.arange(8)[None, :])[0], rtol=1e-13)
