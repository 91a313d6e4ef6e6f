"""Pins for the oracle's local Schwarz part (Sec. 3: overlapping subdomains,
R_p on the interior nodes of bar-Omega_p, A_p = R_p A R_p^T, eq. (asm) local
term), checked by counting, brute force and dense library inverses."""
import numpy as np

from oracle import fem, problem, schwarz
from paper_2606_20496_amd import meshgen as mg


def test_small_cube_restriction_sizes():
    # 8 subdomains of 4^3 elements, one layer of overlap, Dirichlet on x = 0:
    # a subdomain touching x = 0 keeps 4 x 5 x 5 = 100 interior vertices, the
    # others 5 x 5 x 5 = 125 (counting the vertex planes of the extended block).
    m = mg.small_cube()
    sets = schwarz.overlapping_subdomains(m.e2v, m.part, m.n_part, 1)
    R = schwarz.restriction_sets(m.e2v, sets, m.dirichlet)
    assert sorted(len(r) for r in R) == [100] * 4 + [125] * 4
    assert sum(len(r) for r in R) == 900
    assert all(len(s) == 125 for s in sets)   # 5^3 elements after one layer (clipped)


def test_coverage_of_free_vertices():
    m = mg.box_mesh(10, 3, block=3, boxes=(2, 2, 2))
    sets = schwarz.overlapping_subdomains(m.e2v, m.part, m.n_part, 1)
    R = schwarz.restriction_sets(m.e2v, sets, m.dirichlet)
    cover = np.zeros(m.n_vert, int)
    for r in R:
        cover[r] += 1
    free = ~m.dirichlet.astype(bool)
    assert cover[free].min() >= 1 and cover[free].max() <= 8
    assert cover[~free].max() == 0


def _brute_force_sets(e2v, part, n_part, layers, dirichlet):
    # Pure-Python sets, straight from the definitions.
    E = len(e2v)
    ev = [set(map(int, row)) for row in e2v]
    out_R = []
    for p in range(n_part):
        S = {e for e in range(E) if part[e] == p}
        for _ in range(layers):
            verts = set().union(*(ev[e] for e in S))
            S = S | {e for e in range(E) if ev[e] & verts}
        verts = set().union(*(ev[e] for e in S))
        R = sorted(v for v in verts if not dirichlet[v]
                   and all(e in S for e in range(E) if v in ev[e]))
        out_R.append((S, R))
    return out_R


def test_overlap_matches_brute_force():
    for layers in (1, 2):
        m = mg.box_mesh((5, 4, 3), 7, block=2, boxes=(2, 2, 2), faces=("y1",))
        sets = schwarz.overlapping_subdomains(m.e2v, m.part, m.n_part, layers)
        R = schwarz.restriction_sets(m.e2v, sets, m.dirichlet)
        bf = _brute_force_sets(m.e2v, m.part, m.n_part, layers, m.dirichlet)
        for p in range(m.n_part):
            assert set(sets[p].tolist()) == bf[p][0]
            assert R[p].tolist() == bf[p][1]


def test_single_subdomain_is_exact_inverse():
    m = mg.box_mesh(5, 4, block=5, boxes=(1, 1, 1))
    assert m.n_part == 1
    A, Ae, Afull, free, fidx = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
    sets = schwarz.overlapping_subdomains(m.e2v, m.part, m.n_part, 1)
    R = schwarz.restriction_sets(m.e2v, sets, m.dirichlet)
    loc = schwarz.LocalSolves(A, [fidx[r] for r in R])
    r = np.random.default_rng(0).standard_normal(A.shape[0])
    z = loc.apply(r)
    assert np.abs(z - np.linalg.solve(A.toarray(), r)).max() < 1e-12 * np.abs(z).max()


def test_local_part_against_dense_inverses():
    m = mg.box_mesh(6, 5, block=3, boxes=(2, 2, 2), faces=("z0",))
    A, Ae, Afull, free, fidx = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
    sets = schwarz.overlapping_subdomains(m.e2v, m.part, m.n_part, 1)
    R = [fidx[r] for r in schwarz.restriction_sets(m.e2v, sets, m.dirichlet)]
    loc = schwarz.LocalSolves(A, R)
    Ad = A.toarray()
    n = Ad.shape[0]
    Mdense = np.zeros((n, n))
    for Rp in R:
        Rm = np.zeros((len(Rp), n))
        Rm[np.arange(len(Rp)), Rp] = 1.0
        Mdense += Rm.T @ np.linalg.inv(Rm @ Ad @ Rm.T) @ Rm
    rng = np.random.default_rng(1)
    for _ in range(3):
        r = rng.standard_normal(n)
        assert np.abs(loc.apply(r) - Mdense @ r).max() < 1e-12 * np.abs(Mdense @ r).max()
    # symmetric positive definite (overlap covers every free vertex)
    assert np.abs(Mdense - Mdense.T).max() < 1e-12 * np.abs(Mdense).max()
    assert np.linalg.eigvalsh(Mdense)[0] > 0


def test_sampled_local_part_against_dense_inverses():
    # the sampled form used at full size: entries of sum_p R_p^T A_p^-1 R_p r from
    # only the subdomains covering the sampled rows, against dense inverses
    m = mg.box_mesh(9, 6, block=3, boxes=(3, 3, 3), faces=("x1",))
    A, Ae, Afull, free, fidx = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
    sets = schwarz.overlapping_subdomains(m.e2v, m.part, m.n_part, 1)
    R = [fidx[r] for r in schwarz.restriction_sets(m.e2v, sets, m.dirichlet)]
    Ad = A.toarray()
    r = np.random.default_rng(2).standard_normal(Ad.shape[0])
    full = np.zeros(Ad.shape[0])
    for Rp in R:
        full[Rp] += np.linalg.solve(Ad[np.ix_(Rp, Rp)], r[Rp])
    rows = np.random.default_rng(3).choice(Ad.shape[0], 17, replace=False)
    got, which = schwarz.local_part_at(A, R, rows, r)
    assert np.abs(got - full[rows]).max() < 1e-12 * np.abs(full).max()
    assert 0 < len(which) < len(R)          # only the covering subdomains were factored


def _inexact_case():
    m = mg.box_mesh(6, 3, block=3, boxes=(2, 2, 2), faces=("x0",))
    P = problem.from_mesh(m, local_iters=2)
    return m, P


def test_inexact_local_one_step_closed_form():
    # one Jacobi-PCG step from zero: z_p = alpha D^{-1} r_p with
    # alpha = (r, D^{-1} r) / (D^{-1} r, A_p D^{-1} r)
    m, P = _inexact_case()
    loc = schwarz.InexactLocalSolves(P.A, P.R, 1)
    r = np.random.default_rng(3).standard_normal(P.A.shape[0])
    Ad = P.A.toarray()
    ref = np.zeros_like(r)
    for R in P.R:
        Ap = Ad[np.ix_(R, R)]
        g = r[R] / np.diag(Ap)
        ref[R] += (r[R] @ g) / (g @ Ap @ g) * g
    assert np.abs(loc.apply(r) - ref).max() < 1e-13 * np.abs(ref).max()


def test_inexact_local_converges_to_exact():
    # n_p steps of CG reach the exact local solve (finite termination), and the
    # A_p-norm error of the local solve never grows with the number of steps
    m, P = _inexact_case()
    r = np.random.default_rng(4).standard_normal(P.A.shape[0])
    exact = P.local.apply(r) if isinstance(P.local, schwarz.LocalSolves) else \
        schwarz.LocalSolves(P.A, P.R).apply(r)
    nmax = max(len(R) for R in P.R)
    full = schwarz.InexactLocalSolves(P.A, P.R, nmax).apply(r)
    assert np.abs(full - exact).max() < 1e-8 * np.abs(exact).max()
    Ad = P.A.toarray()
    R0 = P.R[0]
    Ap = Ad[np.ix_(R0, R0)]
    xs = np.linalg.solve(Ap, r[R0])
    errs = []
    for k in range(1, 8):
        x = schwarz.InexactLocalSolves.jacobi_pcg(Ap, 1.0 / np.diag(Ap), r[R0], k)
        errs.append(float(np.sqrt((x - xs) @ Ap @ (x - xs))))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 0.5 * errs[0]


def test_inexact_local_is_nonlinear_but_homogeneous():
    # the CG coefficients come from r: M(2r) = 2 M(r), M(r1 + r2) != M(r1) + M(r2)
    m, P = _inexact_case()
    rng = np.random.default_rng(5)
    r1, r2 = rng.standard_normal((2, P.A.shape[0]))
    f = P.local.apply
    assert np.abs(f(2 * r1) - 2 * f(r1)).max() < 1e-13 * np.abs(f(r1)).max()
    assert np.abs(f(r1 + r2) - f(r1) - f(r2)).max() > 1e-6 * np.abs(f(r1)).max()


def test_inexact_local_solves_under_flexible_pcg():
    # with the reduced space of eq. (asm) and flexible CG the solve reaches the
    # tolerance; weaker local solves take more iterations than exact ones
    m = mg.box_mesh(12, 5, block=3, boxes=(4, 4, 4))
    its = {}
    for k in (0, 1, 8):
        P = problem.from_mesh(m, local_iters=k)
        u, info = P.solve(m.b, tol=1e-8, flexible=True)
        assert info["converged"] and info["relres_true"] <= 1.01e-8
        its[k] = info["iters"]
    assert its[0] <= its[8] < its[1]
