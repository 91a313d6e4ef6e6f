"""GPU parity of the block solve (coarse_solve_multi): up to 16 right-hand sides on
one mesh, solved by independent PCG recurrences that share the operator's and the
stored inverses' reads (the dense solves on the matrix cores). Each column is held
to the single-vector bars against the FP64 oracle: one preconditioner application
at 1e-12 (relative, max norm), PCG to 1e-8 with the oracle's iteration count. The
mixed forms (FP32 / FP16-stored inverses, FP32 matrix-core products) are held to
the mixed bars: the same 1e-8 true residual with at most 10% more iterations."""
import math

import numpy as np
import pytest

from oracle import problem
from paper_2606_20496_amd import coarse, meshgen as mg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu(v):
    return torch.tensor(np.asarray(v, dtype=np.float64), device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    coarse.load()


CASES = [
    ("cube8", lambda: mg.small_cube()),
    ("ragged", lambda: mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",))),
    ("annulus", lambda: mg.annulus_mesh(12, 22, block=4, boxes=(3, 3, 3))),
    # operator blocks that sum through incidence lists
    ("reoriented", lambda: mg.reorient(mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",)), 7)),
    # a reduced system of 59 tile rows
    ("big_reduced", lambda: mg.box_mesh((24, 24, 20), 24, block=2, boxes=(12, 12, 10), faces=("x1",))),
]


def _rhs(m, k, seed):
    rng = np.random.default_rng(seed)
    cols = [m.b] + [mg.rhs_bumps(m, seed + j) if j % 2 else rng.standard_normal(m.n_vert) for j in range(1, k)]
    return np.stack(cols)


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_multi_precond_matches_oracle(name, make):
    m = make()
    P = problem.from_mesh(m)
    S = coarse.CoarseSolver.from_mesh(m)
    R = np.random.default_rng(3).standard_normal((5, m.n_vert))
    Z = _np(S.apply_precond_multi(_gpu(R)))
    d = m.dirichlet.astype(bool)
    for j in range(R.shape[0]):
        assert _rel(Z[j], P.apply_precond(R[j])) < 1e-12
        assert np.all(Z[j][d] == 0)


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_multi_solve_matches_oracle(name, make):
    m = make()
    P = problem.from_mesh(m)
    S = coarse.CoarseSolver.from_mesh(m)
    B = _rhs(m, 3, 40)
    U, st = S.solve_multi(_gpu(B), tol=1e-8)
    U = _np(U)
    for j in range(B.shape[0]):
        uo, io = P.solve(B[j], tol=1e-8)
        assert st[j]["status"] == 0 and st[j]["iters"] == io["iters"]
        assert st[j]["relres"] <= 1e-8 and st[j]["relres_true"] <= 1.01e-8
        assert np.linalg.norm(U[j] - uo) / np.linalg.norm(uo) < 1e-9
        assert np.all(U[j][m.dirichlet.astype(bool)] == 0)


@pytest.mark.parametrize("precision", ["mixed", "mixed16"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_multi_solve_mixed(name, make, precision):
    m = make()
    P = problem.from_mesh(m)
    S = coarse.CoarseSolver.from_mesh(m, precision=precision)
    # one application against the single-vector mixed path of the same context
    # (both FP32 products of the same stored inverses, other summation orders)
    R = np.random.default_rng(4).standard_normal((3, m.n_vert))
    Z = _np(S.apply_precond_multi(_gpu(R)))
    for j in range(R.shape[0]):
        assert _rel(Z[j], _np(S.apply_precond(_gpu(R[j])))) < 2e-5
    B = _rhs(m, 3, 45)
    U, st = S.solve_multi(_gpu(B), tol=1e-8)
    U = _np(U)
    for j in range(B.shape[0]):
        uo, io = P.solve(B[j], tol=1e-8)
        assert st[j]["status"] == 0 and st[j]["iters"] <= math.ceil(1.1 * io["iters"])
        assert st[j]["relres_true"] <= 1.05e-8
        assert np.linalg.norm(U[j] - uo) / np.linalg.norm(uo) < 1e-6


def test_multi_columns_independent():
    # 16 columns with a zero column and a repeated one: every column equals,
    # bitwise, the block solve of that column alone; the zero column gives u = 0
    # after no iteration; a repeat gives the same bits
    m = mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",))
    S = coarse.CoarseSolver.from_mesh(m)
    B = _rhs(m, 16, 50)
    B[5] = 0.0
    B[9] = B[2]
    U, st = S.solve_multi(_gpu(B), tol=1e-8)
    U = _np(U)
    assert st[5]["iters"] == 0 and st[5]["status"] == 0 and np.all(U[5] == 0)
    assert np.array_equal(U[9], U[2]) and st[9]["iters"] == st[2]["iters"]
    for j in (0, 2, 7, 15):
        u1, s1 = S.solve_multi(_gpu(B[j:j + 1]), tol=1e-8)
        assert s1[0]["iters"] == st[j]["iters"]
        assert np.array_equal(_np(u1)[0], U[j])
    # and the single-vector solve takes the same iterations to the same solution
    for j in (0, 7):
        u, s = S.solve(_gpu(B[j]), tol=1e-8)
        assert s["iters"] == st[j]["iters"]
        assert np.linalg.norm(_np(u) - U[j]) / np.linalg.norm(U[j]) < 1e-9


def test_multi_rejects_bad_arguments():
    m = mg.small_cube()
    S = coarse.CoarseSolver.from_mesh(m)
    with pytest.raises(ValueError):
        S.solve_multi(torch.zeros((17, m.n_vert), dtype=torch.float64, device="cuda"))
    Sl = coarse.CoarseSolver.from_mesh(m, mode="local_only")
    with pytest.raises(coarse.CoarseError) as ei:
        Sl.apply_precond_multi(torch.zeros((2, m.n_vert), dtype=torch.float64, device="cuda"))
    assert ei.value.code == -1


# ---------------------------------------------------------------------------
# The 64^3 cube (512 subdomains of 8^3): 16 right-hand sides, column 0 the
# benchmark load, against the oracle's solve of it and the oracle's
# preconditioner on four random columns
# ---------------------------------------------------------------------------
@pytest.mark.timeout(900)
def test_multi_cube64():
    m = mg.gpu_share_cube()
    P = problem.from_mesh(m)
    S = coarse.CoarseSolver.from_mesh(m)
    R = np.random.default_rng(13).standard_normal((4, m.n_vert))
    Z = _np(S.apply_precond_multi(_gpu(R)))
    for j in range(4):
        assert _rel(Z[j], P.apply_precond(R[j])) < 1e-12
    B = _rhs(m, 16, 60)
    U, st = S.solve_multi(_gpu(B), tol=1e-8)
    U = _np(U)
    uo, io = P.solve(B[0], tol=1e-8)
    assert st[0]["status"] == 0 and st[0]["iters"] == io["iters"]
    assert np.linalg.norm(U[0] - uo) / np.linalg.norm(uo) < 1e-8
    for j in range(16):
        assert st[j]["status"] == 0 and st[j]["relres_true"] <= 1.01e-8
    for j in (1, 2, 15):
        u, s = S.solve(_gpu(B[j]), tol=1e-8)
        assert s["iters"] == st[j]["iters"]
        assert np.linalg.norm(_np(u) - U[j]) / np.linalg.norm(U[j]) < 1e-8
    # the FP16-stored form on the same block
    S16 = coarse.CoarseSolver.from_mesh(m, precision="mixed16")
    U16, st16 = S16.solve_multi(_gpu(B), tol=1e-8)
    for j in range(16):
        assert st16[j]["status"] == 0 and st16[j]["relres_true"] <= 1.05e-8
        assert st16[j]["iters"] <= math.ceil(1.1 * st[j]["iters"])


def test_multi_stepped_equals_solve_multi():
    # the stepped form (begin, advance, done after a synchronisation, end) gives the
    # block solve's results bit for bit; misuse is refused
    m = mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",))
    for precision in ("fp64", "mixed16"):
        S = coarse.CoarseSolver.from_mesh(m, precision=precision)
        B = _gpu(_rhs(m, 5, 70))
        U0, st0 = S.solve_multi(B, tol=1e-8)
        with pytest.raises(coarse.CoarseError):
            S.multi_advance(2)
        S.multi_begin(B, tol=1e-8)
        with pytest.raises(coarse.CoarseError):
            S.multi_begin(B, tol=1e-8)
        with pytest.raises(coarse.CoarseError):
            S.solve_multi(B, tol=1e-8)
        steps = 0
        while True:
            S.multi_advance(3)
            torch.cuda.synchronize()
            steps += 1
            if S.multi_done():
                break
            assert steps < 1000
        U1, st1 = S.multi_end()
        assert torch.equal(U0, U1)
        assert [s["iters"] for s in st0] == [s["iters"] for s in st1]
        assert all(s["status"] == 0 for s in st1)
        S.close()


@pytest.mark.parametrize("precision", ["mixed", "mixed16"])
@pytest.mark.parametrize("name,make", CASES[:3], ids=[c[0] for c in CASES[:3]])
def test_multi_flexible_beta_matches_single(name, make, precision):
    # the mixed forms take the Polak-Ribiere beta in the block solve as in
    # coarse_solve: one column solved as a block takes the single-vector
    # iteration count (only the summation order inside the dense solves differs)
    m = make()
    S = coarse.CoarseSolver.from_mesh(m, precision=precision)
    assert S.info["precision"] > 0
    _, st1 = S.solve(_gpu(m.b), tol=1e-8)
    _, stm = S.solve_multi(_gpu(m.b[None, :]), tol=1e-8)
    assert stm[0]["iters"] == st1["iters"]
    assert stm[0]["relres"] <= 1e-8
    S.close()


def test_block_rhs_allocates_at_setup():
    # opts.block_rhs: the block solve's vectors are allocated by the setup, so the
    # first block solve leaves the context's device footprint unchanged
    m = mg.small_cube()
    S0 = coarse.CoarseSolver.from_mesh(m)
    S1 = coarse.CoarseSolver.from_mesh(m, block_rhs=1)
    assert S1.device_bytes > S0.device_bytes
    before = S1.device_bytes
    B = _gpu(_rhs(m, 3, 5))
    U1, st1 = S1.solve_multi(B, tol=1e-8)
    assert S1.device_bytes == before
    U0, st0 = S0.solve_multi(B, tol=1e-8)
    assert S0.device_bytes == before
    assert torch.equal(U0, U1)
    S0.close()
    S1.close()
