"""GPU parity of the warm start by projection onto prior solutions (Sec. 5):
coarse_solve_projected over a sequence of right-hand sides against the oracle's
Projection on the same sequence. Per solve: the same PCG iteration count, the
same basis size, the same initial residual ||b - A u_bar|| / ||b||, and solutions
that agree far below the solve tolerance; plus the special cases (a repeated
right-hand side, b = 0, a full basis restarting, a reset, a context without a
basis) and the mixed forms held to the 1e-8 residual."""
import math

import numpy as np
import pytest

from oracle import problem, projection as oproj
from paper_2606_20496_amd import coarse, meshgen as mg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu(v):
    return torch.tensor(np.asarray(v, dtype=np.float64), device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    coarse.load()


MESHES = [
    ("cube8", lambda: mg.small_cube()),
    ("ragged", lambda: mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",))),
    ("annulus", lambda: mg.annulus_mesh(12, 22, block=4, boxes=(3, 3, 3))),
]


def _oracle_sequence(P, bs, L, tol=1e-8, flexible=False):
    proj = oproj.Projection(L)
    out = []
    for b in bs:
        n = len(proj.X)
        u, info = oproj.solve_projected(lambda v: P.A @ v, P.M, P.to_free(b), proj, tol=tol, flexible=flexible)
        out.append((u, info, n))
    return out


@pytest.mark.parametrize("name,make", MESHES, ids=[s[0] for s in MESHES])
def test_projected_sequence_matches_oracle(name, make):
    # L = 3 over 8 solves: the basis fills, restarts from one solution, fills again
    m = make()
    bs = mg.rhs_sequence(m, 31, 8)
    P = problem.from_mesh(m)
    ref = _oracle_sequence(P, bs, 3)
    S = coarse.CoarseSolver.from_mesh(m, projection=3)
    plain = None
    for k, (b, (uo, io, n)) in enumerate(zip(bs, ref)):
        u, st = S.solve_projected(_gpu(b), tol=1e-8)
        u = _np(u)
        assert st["code"] == 0 and st["n_basis"] == n, (k, st, n)
        assert st["iters"] == io["iters"], (k, st["iters"], io["iters"])
        assert abs(st["relres0"] - io["r0_rel"]) <= 1e-7 * io["r0_rel"] + 1e-10, (k, st["relres0"], io["r0_rel"])
        assert st["relres"] <= 1e-8 and st["relres_true"] <= 1.01e-8
        assert np.linalg.norm(u[P.free] - uo) / np.linalg.norm(uo) < 1e-9
        assert np.all(u[m.dirichlet.astype(bool)] == 0)
        if k == 0:
            plain = st["iters"]
    # the warm start pays: later solves need fewer iterations than a cold one
    assert max(r[1]["iters"] for r in ref[2:]) < plain


def test_repeated_rhs_zero_rhs_and_reset():
    # call by call against the oracle: a cold solve, the same b twice (the second
    # starts from the last solution and appends nothing), a new b, b = 0 (u = 0 at
    # once, nothing appended), a reset
    m = mg.small_cube()
    P = problem.from_mesh(m)
    b0, b1 = mg.rhs_sequence(m, 32, 2)
    zero = np.zeros(m.n_vert)
    calls = [("plain", b0), ("proj", b0), ("proj", b0), ("proj", b1), ("proj", zero), ("proj", b1),
             ("reset", None), ("proj", b1)]
    S = coarse.CoarseSolver.from_mesh(m, projection=4)
    proj = oproj.Projection(4)
    last = {}
    for k, (what, b) in enumerate(calls):
        if what == "reset":
            S.projection_reset()
            proj = oproj.Projection(4)
            continue
        if what == "plain":
            u, st = S.solve(_gpu(b), tol=1e-8)
            uo, io = P.solve(b, tol=1e-8)
            uo, n, r0 = uo[P.free], 0, 1.0
        else:
            n = len(proj.X)
            u, st = S.solve_projected(_gpu(b), tol=1e-8)
            uo, io = oproj.solve_projected(lambda v: P.A @ v, P.M, P.to_free(b), proj, tol=1e-8)
            r0 = io["r0_rel"]
        u = _np(u)
        assert st["code"] == 0 and st["n_basis"] == n and st["iters"] == io["iters"], (k, st, io, n)
        assert abs(st["relres0"] - r0) <= 1e-7 * r0 + 1e-10, (k, st["relres0"], r0)
        if what == "plain":
            assert st["relres0"] == 1.0
        if np.any(b):
            assert np.linalg.norm(u[P.free] - uo) / np.linalg.norm(uo) < 1e-9
        else:
            assert not np.any(u)
        last[k] = (u, st)
    # the repeated b needs at most one iteration; the new one fewer than cold
    assert last[2][1]["iters"] <= 1 and last[2][1]["relres0"] <= 1.01e-8
    assert last[3][1]["n_basis"] == 1 and 0 < last[3][1]["iters"] < last[0][1]["iters"]
    # after the reset the projected solve is the plain one, bit for bit
    u7, st7 = last[7]
    u8, st8 = S.solve(_gpu(b1), tol=1e-8)
    assert st7["n_basis"] == 0 and st7["iters"] == st8["iters"] and np.array_equal(u7, _np(u8))


def test_projection_needs_a_basis():
    m = mg.small_cube()
    S = coarse.CoarseSolver.from_mesh(m)
    with pytest.raises(coarse.CoarseError):
        S.solve_projected(_gpu(m.b), tol=1e-8)
    with pytest.raises(coarse.CoarseError):
        coarse.CoarseSolver.from_mesh(m, projection=coarse.PROJECTION_MAX + 1)


def test_projected_sequence_is_bitwise_reproducible():
    m = mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",))
    bs = mg.rhs_sequence(m, 33, 5)
    outs = []
    for _ in range(2):
        S = coarse.CoarseSolver.from_mesh(m, projection=2)
        outs.append([(_np(u), st["iters"]) for u, st in (S.solve_projected(_gpu(b), tol=1e-8) for b in bs)])
        S.close()
    for (ua, ia), (ub, ib) in zip(*outs):
        assert ia == ib and np.array_equal(ua, ub)


@pytest.mark.parametrize("precision", ["mixed", "mixed16"])
def test_projected_sequence_mixed(precision):
    # the basis and the projection stay FP64; the preconditioner is the mixed one
    m = mg.annulus_mesh(12, 22, block=4, boxes=(3, 3, 3))
    bs = mg.rhs_sequence(m, 34, 6)
    P = problem.from_mesh(m)
    ref = _oracle_sequence(P, bs, 4)
    S = coarse.CoarseSolver.from_mesh(m, precision=precision, projection=4)
    for k, (b, (uo, io, n)) in enumerate(zip(bs, ref)):
        u, st = S.solve_projected(_gpu(b), tol=1e-8)
        assert st["code"] == 0 and st["n_basis"] == n
        assert st["iters"] <= math.ceil(1.1 * io["iters"]) + 1, (k, st["iters"], io["iters"])
        assert st["relres_true"] <= 1.05e-8
        assert np.linalg.norm(_np(u)[P.free] - uo) / np.linalg.norm(uo) < 1e-6
