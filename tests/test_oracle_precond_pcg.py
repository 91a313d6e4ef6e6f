"""Pins for the oracle's two-level preconditioner (eq. (asm)) and PCG: dense
library inverses on tiny meshes, symmetry and definiteness, the special case
whose spectrum is known in closed form, textbook CG properties, and the paper's
qualitative claim that both parts of the method are needed (Sec. 5)."""
import numpy as np
import pytest

from oracle import pcg, problem
from paper_2606_20496_amd import meshgen as mg


def _dense_M(P):
    n = P.A.shape[0]
    return np.column_stack([P.M(e) for e in np.eye(n)])


def test_preconditioner_against_dense_formula():
    m = mg.box_mesh(6, 1, block=3, boxes=(2, 2, 2), faces=("y0",))
    P = problem.from_mesh(m)
    Ad = P.A.toarray()
    n = Ad.shape[0]
    Mloc = np.zeros((n, n))
    for Rp in P.R:
        Rm = np.zeros((len(Rp), n))
        Rm[np.arange(len(Rp)), Rp] = 1.0
        Mloc += Rm.T @ np.linalg.inv(Rm @ Ad @ Rm.T) @ Rm
    Jd = P.coarse.J.toarray()
    # A_r itself is pinned in test_oracle_reduced (closed form, triple product)
    Mr = Jd @ np.linalg.inv(P.coarse.Ar) @ Jd.T
    Mdense = _dense_M(P)
    assert np.abs(Mdense - (Mloc + Mr)).max() < 1e-12 * np.abs(Mdense).max()


def test_preconditioner_symmetric_positive_definite():
    m = mg.box_mesh(6, 2, block=3, boxes=(2, 2, 2))
    P = problem.from_mesh(m)
    M = _dense_M(P)
    assert np.abs(M - M.T).max() < 1e-13 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T))[0] > 0
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal((2, M.shape[0]))
    assert abs(x @ P.M(y) - y @ P.M(x)) < 1e-13 * np.abs(P.M(y)).max() * np.linalg.norm(x) * 10


def test_exact_parts_give_one_iteration():
    # One subdomain and one box per element on an unjittered grid: both terms of
    # eq. (asm) equal A^{-1}, so M^{-1} A = 2 I and PCG converges in one step.
    n = 4
    m = mg.box_mesh(n, 0, block=n, boxes=(n, n, n), jitter=0.0)
    P = problem.from_mesh(m)
    M = _dense_M(P)
    assert np.abs(M @ P.A.toarray() - 2 * np.eye(M.shape[0])).max() < 1e-11
    u, info = P.solve(m.b, tol=1e-10)
    assert info["iters"] == 1


def test_pcg_distinct_eigenvalues():
    # Exact-arithmetic CG terminates in at most k steps for k distinct eigenvalues.
    rng = np.random.default_rng(4)
    lam = np.repeat([1.0, 3.0, 7.0, 20.0], 25)
    Q, _ = np.linalg.qr(rng.standard_normal((100, 100)))
    A = Q @ np.diag(lam) @ Q.T
    b = rng.standard_normal(100)
    x, info = pcg.pcg(lambda v: A @ v, lambda v: v, b, tol=1e-10)
    assert info["iters"] <= 4
    assert np.abs(A @ x - b).max() < 1e-8
    x, info = pcg.pcg(lambda v: A @ v, lambda v: np.linalg.solve(A, v), b, tol=1e-10)
    assert info["iters"] == 1


def test_small_cube_solution_against_direct_solve():
    m = mg.small_cube()
    P = problem.from_mesh(m)
    u, info = P.solve(m.b, tol=1e-8)
    Ad = P.A.toarray()
    ustar = np.linalg.solve(Ad, P.to_free(m.b))
    kappa = np.linalg.cond(Ad)
    err = np.linalg.norm(P.to_free(u) - ustar) / np.linalg.norm(ustar)
    assert info["converged"] and info["relres"] <= 1e-8 and info["relres_true"] <= 1.01e-8
    assert err <= kappa * 1e-8
    assert np.all(u[m.dirichlet.astype(bool)] == 0.0)


def test_both_parts_needed():
    # Sec. 5: neither the local solves nor the reduced solve alone give a fast
    # method; together they converge in far fewer iterations.
    m = mg.box_mesh(12, 5, block=3, boxes=(4, 4, 4))
    its = {}
    for mode in ("additive", "local_only", "coarse_only"):
        P = problem.from_mesh(m, mode=mode)
        u, info = P.solve(m.b, tol=1e-8, max_it=300)
        its[mode] = info["iters"] if info["converged"] else 10 ** 6
    assert its["additive"] < its["local_only"]
    assert its["coarse_only"] == 10 ** 6          # rank-deficient: stalls
    assert its["additive"] * 1.5 < its["local_only"]


def test_condition_bounded_under_refinement():
    # Fixed H/delta with h -> 0 (Sec. 3 bounds): kappa(M^{-1}A) estimated from the
    # CG coefficients stays bounded while kappa(A) grows like h^-2.
    ks = []
    for n, block in ((8, 4), (16, 8)):
        m = mg.box_mesh(n, 3, block=block, boxes=(n // block,) * 3)
        P = problem.from_mesh(m)
        u, info = P.solve(m.b, tol=1e-10, record=True)
        lo, hi = pcg.lanczos_condition(info["alphas"], info["betas"])
        ks.append(hi / lo)
    assert ks[1] < 2.0 * ks[0] and ks[1] < 50


def test_hybrid_symmetric_is_symmetric():
    m = mg.box_mesh(6, 2, block=3, boxes=(2, 2, 2))
    P = problem.from_mesh(m, mode="hybrid_sym")
    M = _dense_M(P)
    assert np.abs(M - M.T).max() < 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T))[0] > 0
    u, info = P.solve(m.b)
    Pa = problem.from_mesh(m)
    ua, infoa = Pa.solve(m.b)
    assert info["converged"] and info["iters"] <= infoa["iters"]


def test_zero_rhs():
    m = mg.small_cube()
    P = problem.from_mesh(m)
    u, info = P.solve(np.zeros(m.n_vert))
    assert info["iters"] == 0 and np.all(u == 0)


def test_breakdown_detected():
    with pytest.raises(FloatingPointError):
        pcg.pcg(lambda v: -v, lambda v: v, np.ones(5))


def _dense_parts(P):
    """M_loc and M_r of eq. (asm) from library inverses of the dense matrices."""
    Ad = P.A.toarray()
    n = Ad.shape[0]
    Mloc = np.zeros((n, n))
    for Rp in P.R:
        Rm = np.zeros((len(Rp), n))
        Rm[np.arange(len(Rp)), Rp] = 1.0
        Mloc += Rm.T @ np.linalg.inv(Rm @ Ad @ Rm.T) @ Rm
    Jd = P.coarse.J.toarray()
    Mr = Jd @ np.linalg.inv(P.coarse.Ar) @ Jd.T
    return Ad, Mloc, Mr


def test_hybrid_paper_against_dense_formula():
    # eqs. (asm1)-(asm2): the local solves first, then the reduced solve of the
    # updated residual, z = M_loc r + M_r (r - A M_loc r). Its error propagator
    # is the product (I - M_r A)(I - M_loc A), and it is not symmetric.
    m = mg.box_mesh(6, 1, block=3, boxes=(2, 2, 2), faces=("y0",))
    P = problem.from_mesh(m, mode="hybrid")
    Ad, Mloc, Mr = _dense_parts(P)
    n = Ad.shape[0]
    I = np.eye(n)
    M = _dense_M(P)
    ref = Mloc + Mr @ (I - Ad @ Mloc)
    assert np.abs(M - ref).max() < 1e-12 * np.abs(ref).max()
    E = I - M @ Ad
    assert np.abs(E - (I - Mr @ Ad) @ (I - Mloc @ Ad)).max() < 1e-11
    # the other order (reduced first) is a different operator
    other = Mr + Mloc @ (I - Ad @ Mr)
    assert np.abs(M - other).max() > 1e-3 * np.abs(M).max()
    assert np.abs(M - M.T).max() > 1e-3 * np.abs(M).max()


@pytest.mark.parametrize("case", ["exact_reduced", "exact_local"])
def test_hybrid_paper_exact_parts(case):
    # With an exact reduced space (one box per element of an unjittered grid, so
    # J = I and A_r = A) or an exact local part (one subdomain), the hybrid form
    # is A^{-1} itself; the additive form would give 2 A^{-1} only in the first
    # case and A^{-1} + M_r in the second.
    n = 4
    if case == "exact_reduced":
        m = mg.box_mesh(n, 0, block=2, boxes=(n, n, n), jitter=0.0)
    else:
        m = mg.box_mesh(n, 3, block=n, boxes=(2, 2, 2))
    P = problem.from_mesh(m, mode="hybrid")
    M = _dense_M(P)
    assert np.abs(M @ P.A.toarray() - np.eye(M.shape[0])).max() < 1e-10
    u, info = P.solve(m.b, tol=1e-10, flexible=True)
    assert info["iters"] == 1


def test_hybrid_paper_under_flexible_cg():
    # Under flexible CG the non-symmetric hybrid reaches the same true residual.
    # With the unweighted local sum (each vertex in up to 8 local systems, so
    # lambda_max(M_loc A) = 8) it needs a few more iterations than eq. (asm) here:
    # the hybrid's advantage in the paper is as a single application per cycle.
    m = mg.box_mesh(12, 5, block=3, boxes=(4, 4, 4))
    Pa = problem.from_mesh(m)
    Ph = problem.from_mesh(m, mode="hybrid")
    ua, ia = Pa.solve(m.b, tol=1e-8)
    uh, ih = Ph.solve(m.b, tol=1e-8, flexible=True)
    assert ih["converged"] and ih["relres_true"] <= 1.01e-8
    assert ia["iters"] <= ih["iters"] <= 1.5 * ia["iters"]
    assert np.linalg.norm(uh - ua) <= 1e-6 * np.linalg.norm(ua)


def test_lanczos_condition_recovers_known_spectrum():
    # At termination after k steps on a matrix with k distinct eigenvalues (all
    # present in b), the Lanczos tridiagonal built from the CG coefficients has
    # exactly those eigenvalues; the extremes are returned.
    rng = np.random.default_rng(5)
    lam = np.repeat([0.5, 2.0, 9.0, 40.0], 20)
    Q, _ = np.linalg.qr(rng.standard_normal((lam.size, lam.size)))
    A = Q @ np.diag(lam) @ Q.T
    b = rng.standard_normal(lam.size)
    x, info = pcg.pcg(lambda v: A @ v, lambda v: v, b, tol=1e-10, record=True)
    assert info["iters"] == 4
    lo, hi = pcg.lanczos_condition(info["alphas"], info["betas"])
    assert abs(lo - 0.5) < 1e-9 and abs(hi - 40.0) < 1e-8
    # preconditioned: B commutes with A, so M^{-1}A = B A has eigenvalues mu * lam
    mu = np.repeat([4.0, 1.5, 1.0, 0.1], 20)            # mu * lam = 2, 3, 9, 4
    B = Q @ np.diag(mu) @ Q.T
    x, info = pcg.pcg(lambda v: A @ v, lambda v: B @ v, b, tol=1e-10, record=True)
    lo, hi = pcg.lanczos_condition(info["alphas"], info["betas"])
    assert info["iters"] == 4
    assert abs(lo - 2.0) < 1e-9 and abs(hi - 9.0) < 1e-8
    # before termination the estimates lie inside the spectrum (Ritz values)
    x, info = pcg.pcg(lambda v: A @ v, lambda v: v, b, tol=1e-13, max_it=2, record=True)
    lo, hi = pcg.lanczos_condition(info["alphas"], info["betas"][:1])
    assert 0.5 - 1e-12 <= lo <= hi <= 40.0 + 1e-12
