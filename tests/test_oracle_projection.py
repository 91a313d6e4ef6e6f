"""Pins for the oracle's projection onto prior solutions (Sec. 5: the initial
guess is the A-orthogonal best fit of the new solution in the span of prior
solutions), against the closed form of that projection and its invariants."""
import numpy as np

from oracle import fem, projection, problem
from paper_2606_20496_amd import meshgen as mg


def _system():
    m = mg.box_mesh(6, 61, block=3, boxes=(2, 2, 2))
    A, _, _, free, _ = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
    return m, A.toarray(), free


def test_basis_is_a_orthonormal_and_guess_is_the_best_fit():
    m, A, free = _system()
    rng = np.random.default_rng(3)
    proj = projection.Projection(5)
    U = []
    for _ in range(4):
        u = rng.standard_normal(A.shape[0])
        U.append(u)
        proj.add(u, A @ u)
    X = np.array(proj.X).T
    assert np.abs(X.T @ A @ X - np.eye(4)).max() < 1e-10
    # best fit in the A-norm over span(U): (U^T A U) c = U^T b
    b = rng.standard_normal(A.shape[0])
    Um = np.array(U).T
    c = np.linalg.solve(Um.T @ A @ Um, Um.T @ b)
    ubar, r0 = proj.initial_guess(b)
    assert np.abs(ubar - Um @ c).max() < 1e-9 * np.abs(Um @ c).max()
    assert np.abs(r0 - (b - A @ ubar)).max() < 1e-9 * np.abs(b).max()
    # the remainder is A-orthogonal to the span: U^T r0 = 0
    assert np.abs(Um.T @ r0).max() < 1e-9 * np.abs(Um.T @ b).max()


def test_repeated_right_hand_side_needs_no_iteration_and_restart():
    m = mg.box_mesh(6, 62, block=3, boxes=(2, 2, 2))
    P = problem.from_mesh(m)
    proj = projection.Projection(2)
    b = P.to_free(m.b)
    u1, i1 = projection.solve_projected(lambda v: P.A @ v, P.M, b, proj, tol=1e-8)
    assert i1["iters"] > 0 and len(proj.X) == 1
    u2, i2 = projection.solve_projected(lambda v: P.A @ v, P.M, b, proj, tol=1e-8)
    assert i2["iters"] == 0 and np.abs(u2 - u1).max() < 1e-7 * np.abs(u1).max()
    # the third solution fills the basis (2), the fourth restarts it
    b3 = b + 0.1 * np.random.default_rng(4).standard_normal(b.size)
    projection.solve_projected(lambda v: P.A @ v, P.M, b3, proj, tol=1e-8)
    projection.solve_projected(lambda v: P.A @ v, P.M, 2 * b3, proj, tol=1e-8)
    assert len(proj.X) == 1


def test_projected_solve_reaches_the_tolerance_of_b():
    m = mg.box_mesh(8, 63, block=4, boxes=(2, 2, 2))
    P = problem.from_mesh(m)
    proj = projection.Projection(4)
    b0 = P.to_free(m.b)
    rng = np.random.default_rng(5)
    iters = []
    for k in range(5):
        b = b0 + 0.05 * k * rng.standard_normal(b0.size)
        u, info = projection.solve_projected(lambda v: P.A @ v, P.M, b, proj, tol=1e-8)
        assert np.linalg.norm(b - P.A @ u) <= 1.01e-8 * np.linalg.norm(b)
        iters.append(info["iters"])
    assert min(iters[1:]) < iters[0]
