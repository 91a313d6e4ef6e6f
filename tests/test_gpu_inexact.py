"""GPU parity of the inexact local solves (k steps of Jacobi-preconditioned CG
per subdomain in place of A_p^{-1}) against the oracle's InexactLocalSolves on the
same seeded inputs. Bars as for the exact solves: one FP64 preconditioner
application at 1e-12 (relative, max norm), flexible PCG to 1e-8 with the oracle's
iteration count; FP32-stored A_p (mixed forms) reaches the same 1e-8 residual
within max(ceil(1.1 k), k + 2) iterations of the oracle's k."""
import math

import numpy as np
import pytest

from iteration_bar import check_fp64_iters
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


SMALL = [
    ("cube8", lambda: mg.small_cube()),
    ("ragged", lambda: mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",))),
    ("annulus", lambda: mg.annulus_mesh(12, 22, block=4, boxes=(3, 3, 3))),
    ("one_sub", lambda: mg.box_mesh(6, 23, block=6, boxes=(2, 2, 2), faces=("z0",))),
    ("reoriented", lambda: mg.reorient(mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",)), 7)),
    ("big_reduced", lambda: mg.box_mesh((24, 24, 20), 24, block=2, boxes=(12, 12, 10), faces=("x1",))),
]


@pytest.mark.parametrize("k", [1, 3, 8])
@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_inexact_apply_matches_oracle(name, make, k):
    m = make()
    P = problem.from_mesh(m, local_iters=k)
    S = coarse.CoarseSolver.from_mesh(m, local_iters=k)
    assert S.info["local_iters"] == k and 0 < S.info["ell_width"] <= 26
    rng = np.random.default_rng(40 + k)
    for _ in range(2):
        r = rng.standard_normal(m.n_vert)
        z = _np(S.apply_precond(_gpu(r)))
        assert _rel(z, P.apply_precond(r)) < 1e-12
        assert np.all(z[m.dirichlet.astype(bool)] == 0)


@pytest.mark.parametrize("k", [2, 6])
@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_inexact_solve_matches_oracle(name, make, k):
    m = make()
    P = problem.from_mesh(m, local_iters=k)
    S = coarse.CoarseSolver.from_mesh(m, local_iters=k)
    uo, io = P.solve(m.b, tol=1e-8, flexible=True)
    u, st = S.solve(_gpu(m.b), tol=1e-8)
    assert st["code"] == 0 and st["iters"] == io["iters"]
    assert st["relres_true"] <= 1.01e-8
    assert np.linalg.norm(_np(u) - uo) / np.linalg.norm(uo) < 1e-9


@pytest.mark.parametrize("mode", ["local_only", "hybrid", "hybrid_sym"])
def test_inexact_other_modes(mode):
    m = mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",))
    P = problem.from_mesh(m, local_iters=3, mode=mode)
    S = coarse.CoarseSolver.from_mesh(m, local_iters=3, mode=mode)
    r = np.random.default_rng(47).standard_normal(m.n_vert)
    assert _rel(_np(S.apply_precond(_gpu(r))), P.apply_precond(r)) < 1e-12


def test_inexact_many_steps_equal_exact_solves():
    # k >= |R_p| CG steps solve each local system exactly (finite termination, up
    # to rounding): the inexact preconditioner then equals the exact one
    m = mg.small_cube()
    S_ex = coarse.CoarseSolver.from_mesh(m)
    S_in = coarse.CoarseSolver.from_mesh(m, local_iters=int(S_ex.info["max_np"]) + 5)
    r = np.random.default_rng(48).standard_normal(m.n_vert)
    z_ex = _np(S_ex.apply_precond(_gpu(r)))
    assert _rel(_np(S_in.apply_precond(_gpu(r))), z_ex) < 1e-9


@pytest.mark.parametrize("precision", ["mixed", "mixed16"])
@pytest.mark.parametrize("name,make", SMALL[:4], ids=[s[0] for s in SMALL[:4]])
def test_inexact_mixed(name, make, precision):
    m = make()
    k = 4
    P = problem.from_mesh(m, local_iters=k)
    _, io = P.solve(m.b, tol=1e-8, flexible=True)
    S = coarse.CoarseSolver.from_mesh(m, local_iters=k, precision=precision)
    u, st = S.solve(_gpu(m.b), tol=1e-8)
    assert st["code"] == 0 and st["relres_true"] <= 1.01e-8
    assert st["iters"] <= max(math.ceil(1.1 * io["iters"]), io["iters"] + 2)


def test_inexact_repeat_is_bitwise_and_zero_rhs():
    m = mg.annulus_mesh(12, 22, block=4, boxes=(3, 3, 3))
    S = coarse.CoarseSolver.from_mesh(m, local_iters=5)
    r = _gpu(np.random.default_rng(49).standard_normal(m.n_vert))
    z1 = _np(S.apply_precond(r))
    z2 = _np(S.apply_precond(r))
    assert np.array_equal(z1, z2)
    assert np.all(_np(S.apply_precond(_gpu(np.zeros(m.n_vert)))) == 0)
    u1, _ = S.solve(_gpu(m.b))
    u2, _ = S.solve(_gpu(m.b))
    assert torch.equal(u1, u2)


def test_inexact_projected_solves():
    # the projected initial guess (Sec. 5) works with inexact local solves: a
    # repeated right-hand side converges at once, a new one from a smaller residual
    m = mg.box_mesh(8, 33, block=4, boxes=(2, 2, 2))
    S = coarse.CoarseSolver.from_mesh(m, local_iters=4, projection=4)
    b = _gpu(m.b)
    u1, st1 = S.solve_projected(b)
    u2, st2 = S.solve_projected(b)
    assert st1["code"] == 0 and st2["code"] == 0
    assert st2["iters"] <= 1 and st2["relres_true"] <= 1.01e-8


def test_inexact_rejected_where_unsupported():
    m = mg.small_cube()
    S = coarse.CoarseSolver.from_mesh(m, local_iters=2)
    with pytest.raises(coarse.CoarseError):
        S.solve_multi(torch.stack([_gpu(m.b), _gpu(m.b)], 0))
    # subdomains of more than 1024 free vertices
    big = mg.box_mesh(20, 34, block=10, boxes=(2, 2, 2))
    with pytest.raises(coarse.CoarseError) as ei:
        coarse.CoarseSolver.from_mesh(big, local_iters=2)
    assert ei.value.code == -1


@pytest.mark.timeout(900)
def test_inexact_cube64():
    # one GPU's share (64^3, 512 subdomains of 8^3 elements): one application at
    # 1e-12 and the oracle's flexible iteration count
    m = mg.gpu_share_cube()
    k = 4
    P = problem.from_mesh(m, local_iters=k)
    S = coarse.CoarseSolver.from_mesh(m, local_iters=k)
    r = np.random.default_rng(50).standard_normal(m.n_vert)
    assert _rel(_np(S.apply_precond(_gpu(r))), P.apply_precond(r)) < 1e-12
    _, io = P.solve(m.b, tol=1e-8, flexible=True)
    u, st = S.solve(_gpu(m.b), tol=1e-8)
    assert st["code"] == 0 and st["iters"] == io["iters"] and st["relres_true"] <= 1.01e-8


def _batch_case(precision):
    # batch-workload meshes (n <= 24, blocks of 4, 6 or 8 elements); every other
    # context uses inexact local solves, with different step counts
    ms = mg.batch_meshes(count=8, nmax=24)
    kw = [dict(local_iters=(0 if j % 2 else 2 + j)) for j in range(len(ms))]
    return ms, kw


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("graph", [False, True])
def test_inexact_in_batch_equals_alone(precision, graph):
    # the grouped launch of the inexact local solves (one workgroup size for all
    # solves) gives bitwise the solve alone, beside exact-solve contexts
    ms, kw = _batch_case(precision)
    ref = []
    for m, k in zip(ms, kw):
        S = coarse.CoarseSolver.from_mesh(m, precision=precision, **k)
        u, st = S.solve(_gpu(m.b))
        ref.append((u, st["iters"]))
    solvers = [coarse.CoarseSolver.from_mesh(m, precision=precision, **k) for m, k in zip(ms, kw)]
    bs = [_gpu(m.b) for m in ms]
    us = [torch.zeros_like(b) for b in bs]
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    bt = coarse.Batch(stream=stream, use_graph=graph)
    done = {}
    for j in range(4):
        bt.submit(solvers[j], bs[j], us[j], tag=j)
    for tag, st in bt.step(3):
        done[tag] = st
    for j in range(4, len(ms)):
        bt.submit(solvers[j], bs[j], us[j], tag=j)
    guard = 0
    while bt.live > 0:
        for tag, st in bt.step(2):
            done[tag] = st
        guard += 1
        assert guard < 1000
    stream.synchronize()
    for j in range(len(ms)):
        assert done[j]["code"] == 0 and done[j]["iters"] == ref[j][1]
        assert torch.equal(us[j], ref[j][0]), j
    bt.close()


def test_inexact_batch_matches_oracle_and_noalloc():
    ms, kw = _batch_case("fp64")
    ms, kw = ms[:4], kw[:4]
    solvers = [coarse.CoarseSolver.from_mesh(m, **k) for m, k in zip(ms, kw)]
    bs = [_gpu(m.b) for m in ms]
    us, sts = coarse.solve_batch(solvers, bs)
    us2, sts2 = coarse.solve_batch(solvers, bs, noalloc=True)
    for m, k, u, u2, st, st2 in zip(ms, kw, us, us2, sts, sts2):
        P = problem.from_mesh(m, **k)
        uo, io = P.solve(m.b, tol=1e-8, flexible=k["local_iters"] > 0)
        check_fp64_iters(st["iters"], P, m.b, io["iters"], flexible=k["local_iters"] > 0)
        assert st2["iters"] == st["iters"]
        assert torch.equal(u, u2)
        # i.i.d. right-hand sides on the batch meshes: the 1e-7 bar of those meshes
        assert np.linalg.norm(_np(u) - uo) / np.linalg.norm(uo) < 1e-7


@pytest.mark.parametrize("precision", ["mixed", "mixed16"])
def test_inexact_mixed_application_error(precision):
    # the mixed forms store A_p in FP32 and run the local CG in FP32: one
    # application against the FP64 oracle of the same k, relative, max norm. The
    # local CG's FP32 rounding (k steps, a few dozen operations per value) sits
    # far below 1e-4; the reduced term keeps its FP32 / FP16-storage error
    m = mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",))
    errs = {}
    for k in (2, 6):
        P = problem.from_mesh(m, local_iters=k)
        S = coarse.CoarseSolver.from_mesh(m, local_iters=k, precision=precision)
        r = np.random.default_rng(70 + k).standard_normal(m.n_vert)
        errs[k] = _rel(_np(S.apply_precond(_gpu(r))), P.apply_precond(r))
    print(f"{precision} inexact application error vs FP64 oracle: {errs}")
    assert max(errs.values()) < (1e-4 if precision == "mixed" else 4 * 2.0 ** -11)
