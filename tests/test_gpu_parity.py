"""GPU parity: the HIP path through the C-ABI against the FP64 oracle on the same
seeded inputs. Bars: A apply 1e-13 and one preconditioner application 1e-12
(relative, max norm) in FP64; PCG to 1e-8 with the same iteration count. Mixed
precision: the same 1e-8 residual with at most 10% more iterations."""
import math

import numpy as np
import pytest

from oracle import pcg as opcg, precond as oprec, problem
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


def _case(m, **kw):
    P = problem.from_mesh(m, **{k: v for k, v in kw.items() if k in ("overlap", "mode")})
    S = coarse.CoarseSolver.from_mesh(m, **kw)
    return P, S


SMALL = [
    ("cube8", lambda: mg.small_cube()),
    ("ragged", lambda: mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",))),
    ("annulus", lambda: mg.annulus_mesh(12, 22, block=4, boxes=(3, 3, 3))),
    ("one_sub", lambda: mg.box_mesh(6, 23, block=6, boxes=(2, 2, 2), faces=("z0",))),
    # elements of mixed local orientation: operator blocks sum through incidence lists
    ("reoriented", lambda: mg.reorient(mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",)), 7)),
    # 1859 reduced unknowns (59 tile rows): the reduced branch runs on a second stream
    ("big_reduced", lambda: mg.box_mesh((24, 24, 20), 24, block=2, boxes=(12, 12, 10), faces=("x1",))),
]


def test_reduced_branch_stream_choice():
    # a reduced system of more than 48 tile rows is solved on the second stream
    # (profile phase 7, no separate corner-sum phase); a smaller one shares the
    # dense-solve launch of the local systems
    for make, aside in ((SMALL[-1][1], 1), (mg.small_cube, 0)):
        m = make()
        S = coarse.CoarseSolver.from_mesh(m)
        assert S.info["reduced_stream"] == aside
        S.profile_start()
        S.apply_precond(_gpu(np.ones(m.n_vert)))
        ph = S.profile_stop()
        assert ph[coarse.PHASES[7]][1] == aside and ph[coarse.PHASES[2]][1] == 1 - aside
        assert ph[coarse.PHASES[3]][1] == 1


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_apply_A_small(name, make):
    m = make()
    P, S = _case(m)
    rng = np.random.default_rng(5)
    for _ in range(2):
        p = rng.standard_normal(m.n_vert)
        q = _np(S.apply_A(_gpu(p)))
        assert _rel(q, P.apply_A(p)) < 1e-13
        assert np.all(q[m.dirichlet.astype(bool)] == 0)


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_apply_precond_small(name, make):
    m = make()
    P, S = _case(m)
    rng = np.random.default_rng(6)
    for _ in range(2):
        r = rng.standard_normal(m.n_vert)
        z = _np(S.apply_precond(_gpu(r)))
        assert _rel(z, P.apply_precond(r)) < 1e-12
        assert np.all(z[m.dirichlet.astype(bool)] == 0)


@pytest.mark.parametrize("mode", ["local_only", "reduced_only", "hybrid_sym", "hybrid"])
def test_apply_precond_modes(mode):
    m = mg.box_mesh(8, 31, block=4, boxes=(2, 2, 2), faces=("x0", "z1"))
    om = {"reduced_only": "coarse_only"}.get(mode, mode)
    P = problem.from_mesh(m, mode=om)
    S = coarse.CoarseSolver.from_mesh(m, mode=mode)
    r = np.random.default_rng(7).standard_normal(m.n_vert)
    assert _rel(_np(S.apply_precond(_gpu(r))), P.apply_precond(r)) < 1e-12


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_standard_interp_precond_and_solve(name, make):
    # vertex-based J with the Galerkin A_r = J^T A J (Sec. 4), formed on the GPU
    # by probes: one preconditioner application at 1e-12, the same iterations
    m = make()
    P = problem.from_mesh(m, interp="standard")
    S = coarse.CoarseSolver.from_mesh(m, interp="standard")
    r = np.random.default_rng(10).standard_normal(m.n_vert)
    assert _rel(_np(S.apply_precond(_gpu(r))), P.apply_precond(r)) < 1e-12
    uo, io = P.solve(m.b, tol=1e-8)
    u, st = S.solve(_gpu(m.b), tol=1e-8)
    assert st["code"] == 0 and st["iters"] == io["iters"]
    assert np.linalg.norm(_np(u) - uo) / np.linalg.norm(uo) < 1e-9


def test_standard_interp_reduced_part_is_a_projection():
    # with A_r = J^T A J, z = J A_r^{-1} J^T r is the A-orthogonal projection of
    # A^{-1} r on range(J): J^T (r - A z) = 0 (the best-approximation property)
    m = mg.box_mesh(12, 44, block=4, boxes=(3, 3, 3), faces=("z0",))
    P = problem.from_mesh(m, interp="standard")
    S = coarse.CoarseSolver.from_mesh(m, interp="standard", mode="reduced_only")
    r = np.random.default_rng(11).standard_normal(m.n_vert)
    z = S.apply_precond(_gpu(r))
    q = _np(S.apply_A(z))
    J = P.coarse.J
    res = J.T @ (P.to_free(r) - P.to_free(q))
    assert np.abs(res).max() < 1e-11 * np.abs(J.T @ P.to_free(r)).max()


@pytest.mark.parametrize("mode", ["hybrid_sym", "local_only", "hybrid"])
def test_solve_modes_match_oracle(mode):
    # the whole PCG loop with the symmetrised hybrid, the paper's hybrid of eqs.
    # (asm1)-(asm2) (not symmetric: flexible beta on both sides) and the local part
    # alone: the same iterations as the oracle and the same solution to the tolerance
    m = mg.box_mesh(12, 47, block=4, boxes=(3, 3, 3), faces=("x0",), rhs="bumps")
    om = {"reduced_only": "coarse_only"}.get(mode, mode)
    P = problem.from_mesh(m, mode=om)
    uo, io = P.solve(m.b, tol=1e-8, flexible=(mode == "hybrid"))
    S = coarse.CoarseSolver.from_mesh(m, mode=mode)
    u, st = S.solve(_gpu(m.b), tol=1e-8)
    assert st["code"] == 0 and st["iters"] == io["iters"]
    assert np.linalg.norm(_np(u) - uo) / np.linalg.norm(uo) < 1e-9


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_hybrid_paper_small(name, make):
    # eqs. (asm1)-(asm2) as written: one application at 1e-12 against the oracle,
    # and flexible PCG with the oracle's iteration count
    m = make()
    P = problem.from_mesh(m, mode="hybrid")
    S = coarse.CoarseSolver.from_mesh(m, mode="hybrid")
    r = np.random.default_rng(15).standard_normal(m.n_vert)
    assert _rel(_np(S.apply_precond(_gpu(r))), P.apply_precond(r)) < 1e-12
    uo, io = P.solve(m.b, tol=1e-8, flexible=True)
    u, st = S.solve(_gpu(m.b), tol=1e-8)
    assert st["code"] == 0 and st["iters"] == io["iters"]
    assert st["relres_true"] <= 1.01e-8
    assert np.linalg.norm(_np(u) - uo) / np.linalg.norm(uo) < 1e-9


def test_overlap_two():
    m = mg.box_mesh(8, 32, block=4, boxes=(2, 2, 2))
    P, S = _case(m, overlap=2)
    r = np.random.default_rng(8).standard_normal(m.n_vert)
    assert _rel(_np(S.apply_precond(_gpu(r))), P.apply_precond(r)) < 1e-12


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_solve_small_fp64(name, make):
    m = make()
    P, S = _case(m)
    uo, io = P.solve(m.b, tol=1e-8)
    u, st = S.solve(_gpu(m.b), tol=1e-8)
    u = _np(u)
    assert st["code"] == 0 and st["iters"] == io["iters"]
    assert st["relres"] <= 1e-8 and st["relres_true"] <= 1.01e-8
    # both iterates agree far below the solve tolerance
    assert np.linalg.norm(u - uo) / np.linalg.norm(uo) < 1e-9
    assert np.all(u[m.dirichlet.astype(bool)] == 0)


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_solve_small_mixed(name, make):
    m = make()
    P = problem.from_mesh(m)
    uo, io = P.solve(m.b, tol=1e-8)
    S = coarse.CoarseSolver.from_mesh(m, precision="mixed")
    u, st = S.solve(_gpu(m.b), tol=1e-8)
    assert st["code"] == 0
    assert st["iters"] <= math.ceil(1.1 * io["iters"])
    assert st["relres_true"] <= 1.05e-8
    assert np.linalg.norm(_np(u) - uo) / np.linalg.norm(uo) < 1e-6


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_solve_small_mixed16(name, make):
    # FP16 storage of the inverses (per-system power-of-two scale), FP32 arithmetic.
    # A reduced-byte form of the local solves is weighed by iterations x bytes: it
    # must reach the same 1e-8 true residual and move no more bytes through the
    # dense solves than the FP32 form (at most twice its iterations)
    m = make()
    P = problem.from_mesh(m)
    uo, io = P.solve(m.b, tol=1e-8)
    S = coarse.CoarseSolver.from_mesh(m, precision="mixed16")
    S32 = coarse.CoarseSolver.from_mesh(m, precision="mixed")
    assert S.info["inv_alg_bytes"] * 2 == S32.info["inv_alg_bytes"]
    u, st = S.solve(_gpu(m.b), tol=1e-8)
    _, st32 = S32.solve(_gpu(m.b), tol=1e-8)
    assert st["code"] == 0
    assert st["iters"] * S.info["inv_alg_bytes"] <= st32["iters"] * S32.info["inv_alg_bytes"]
    assert st["relres_true"] <= 1.05e-8
    assert np.linalg.norm(_np(u) - uo) / np.linalg.norm(uo) < 1e-6


def test_zero_rhs_and_dirichlet_entries_ignored():
    m = mg.small_cube()
    S = coarse.CoarseSolver.from_mesh(m)
    u, st = S.solve(_gpu(np.zeros(m.n_vert)))
    assert st["iters"] == 0 and float(u.abs().max()) == 0.0
    b = m.b.copy()
    b[m.dirichlet.astype(bool)] = 1e6
    u1, _ = S.solve(_gpu(m.b))
    u2, _ = S.solve(_gpu(b))
    assert torch.equal(u1, u2)


def test_repeat_is_bitwise():
    m = mg.box_mesh(12, 33, block=4, boxes=(3, 3, 3))
    S = coarse.CoarseSolver.from_mesh(m)
    b = _gpu(m.b)
    u1, s1 = S.solve(b)
    u2, s2 = S.solve(b)
    assert torch.equal(u1, u2) and s1["iters"] == s2["iters"]
    z1 = S.apply_precond(b)
    z2 = S.apply_precond(b)
    assert torch.equal(z1, z2)


def test_check_interval_does_not_change_result():
    m = mg.box_mesh(10, 34, block=5, boxes=(2, 2, 2))
    b = _gpu(m.b)
    outs = []
    for ce in (1, 3, 16):
        S = coarse.CoarseSolver.from_mesh(m, check_every=ce)
        u, st = S.solve(b)
        outs.append((u, st["iters"]))
    assert all(torch.equal(outs[0][0], o[0]) and outs[0][1] == o[1] for o in outs)


def test_iteration_limit_and_breakdown_codes():
    m = mg.small_cube()
    S = coarse.CoarseSolver.from_mesh(m, max_it=3)
    u, st = S.solve(_gpu(m.b))
    assert st["code"] == 1 and st["iters"] == 3
    bad = m.b.copy()
    bad[np.flatnonzero(~m.dirichlet.astype(bool))[0]] = np.nan
    S2 = coarse.CoarseSolver.from_mesh(m)
    with pytest.raises(coarse.CoarseError) as ei:
        S2.solve(_gpu(bad))
    assert ei.value.code == -6
    u, st = S2.solve(_gpu(m.b))          # the context stays usable
    assert st["code"] == 0


def test_setup_errors():
    m = mg.small_cube()
    # all-Neumann: A is singular, the local systems touching nothing Dirichlet are
    # still SPD but the reduced system is not
    with pytest.raises(coarse.CoarseError) as ei:
        coarse.CoarseSolver(m.xyz, m.e2v, np.zeros(m.n_vert, np.uint8), m.part, m.n_part, boxes=m.boxes)
    assert ei.value.code == -4
    # inverted element
    e2v = m.e2v.copy()
    e2v[5] = e2v[5][[1, 0, 3, 2, 5, 4, 7, 6]]
    with pytest.raises(coarse.CoarseError) as ei:
        coarse.CoarseSolver(m.xyz, e2v, m.dirichlet, m.part, m.n_part, boxes=m.boxes)
    assert ei.value.code == -3


# ---------------------------------------------------------------------------
# One GPU's share: the 64^3 cube with 512 subdomains (the benchmark workload)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def cube64():
    m = mg.gpu_share_cube()
    P = problem.from_mesh(m)
    uo, io = P.solve(m.b, tol=1e-8)
    return m, P, uo, io


@pytest.mark.timeout(900)
def test_cube64_precond_and_A(cube64):
    m, P, uo, io = cube64
    S = coarse.CoarseSolver.from_mesh(m)
    r = np.random.default_rng(9).standard_normal(m.n_vert)
    assert _rel(_np(S.apply_A(_gpu(r))), P.apply_A(r)) < 1e-13
    assert _rel(_np(S.apply_precond(_gpu(r))), P.apply_precond(r)) < 1e-12


@pytest.mark.timeout(900)
def test_cube64_solve_fp64(cube64):
    m, P, uo, io = cube64
    S = coarse.CoarseSolver.from_mesh(m)
    u, st = S.solve(_gpu(m.b), tol=1e-8)
    assert st["code"] == 0 and st["iters"] == io["iters"]
    assert st["relres_true"] <= 1.01e-8
    assert np.linalg.norm(_np(u) - uo) / np.linalg.norm(uo) < 1e-8


@pytest.mark.timeout(900)
def test_cube64_solve_mixed16(cube64):
    m, P, uo, io = cube64
    S = coarse.CoarseSolver.from_mesh(m, precision="mixed16")
    u, st = S.solve(_gpu(m.b), tol=1e-8)
    assert st["code"] == 0
    assert st["iters"] <= math.ceil(1.1 * io["iters"])
    assert st["relres_true"] <= 1.05e-8
    assert np.linalg.norm(_np(u) - uo) / np.linalg.norm(uo) < 1e-6


@pytest.mark.timeout(900)
def test_cube64_solve_mixed(cube64):
    m, P, uo, io = cube64
    S = coarse.CoarseSolver.from_mesh(m, precision="mixed")
    u, st = S.solve(_gpu(m.b), tol=1e-8)
    assert st["code"] == 0
    assert st["iters"] <= math.ceil(1.1 * io["iters"])
    assert st["relres_true"] <= 1.05e-8
    assert np.linalg.norm(_np(u) - uo) / np.linalg.norm(uo) < 1e-6


# Error of one mixed-precision preconditioner application against the FP64 oracle
# (relative, max norm), in full on the 8^3 and 64^3 cubes: at most 16 FP32 unit
# roundoffs (2^-24) with FP32 inverses and J, at most 4 FP16 unit roundoffs
# (2^-11) with FP16-stored inverses (each entry of A_p^{-1} is rounded once to
# that precision; the sums and J run in FP32).
MIXED_PRECOND_BAR = {"mixed": 16 * 2.0 ** -24, "mixed16": 4 * 2.0 ** -11}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["mixed", "mixed16"])
def test_mixed_precond_error_vs_oracle(cube64, precision):
    errs = {}
    r = np.random.default_rng(16).standard_normal
    for name, (m, P) in (("cube8", (mg.small_cube(), None)), ("cube64", (cube64[0], cube64[1]))):
        P = problem.from_mesh(m) if P is None else P
        S = coarse.CoarseSolver.from_mesh(m, precision=precision)
        rv = r(m.n_vert)
        errs[name] = _rel(_np(S.apply_precond(_gpu(rv))), P.apply_precond(rv))
        S.close()
    print(f"{precision} preconditioner error vs oracle: {errs}")
    assert max(errs.values()) < MIXED_PRECOND_BAR[precision]


@pytest.mark.timeout(900)
def test_leftover_reduced_system():
    # 320 subdomains, 256 of them with 21-23 tile rows, and a reduced system of 16
    # tile rows: 257 candidates for one workgroup each, so on a 256-unit device the
    # smallest (the reduced system) is past the last full round and goes to work
    # items in the same launch, whose partial sums the combine pass adds and
    # scatters to the box grid
    m = mg.box_mesh((64, 64, 36), 71, block=8, boxes=(8, 8, 5), faces=("z0",))
    P = problem.from_mesh(m)
    S = coarse.CoarseSolver.from_mesh(m)
    r = np.random.default_rng(14).standard_normal(m.n_vert)
    assert _rel(_np(S.apply_precond(_gpu(r))), P.apply_precond(r)) < 1e-12
    uo, io = P.solve(m.b, tol=1e-8)
    u, st = S.solve(_gpu(m.b), tol=1e-8)
    assert st["code"] == 0 and st["iters"] == io["iters"]
    assert np.linalg.norm(_np(u) - uo) / np.linalg.norm(uo) < 1e-9
    S16 = coarse.CoarseSolver.from_mesh(m, precision="mixed16")
    u16, st16 = S16.solve(_gpu(m.b), tol=1e-8)
    assert st16["code"] == 0 and st16["relres_true"] <= 1.05e-8


@pytest.mark.timeout(900)
def test_whole_waves_change_rounding_only(cube64):
    # the wavefront count of the whole-system workgroups (a tuned choice) changes
    # only the order of rounding: every choice meets the 1e-12 preconditioner bar
    # and the oracle's iteration count
    m, P, uo, io = cube64
    r = np.random.default_rng(17).standard_normal(m.n_vert)
    zo = P.apply_precond(r)
    for precision, waves in (("fp64", (2, 4, 8)), ("mixed16", (4, 8, 16))):
        for w in waves:
            S = coarse.CoarseSolver.from_mesh(m, precision=precision, whole_waves=w)
            assert S.info["whole_waves"] == w
            z = _np(S.apply_precond(_gpu(r)))
            u, st = S.solve(_gpu(m.b), tol=1e-8)
            S.close()
            if precision == "fp64":
                assert _rel(z, zo) < 1e-12, w
                assert st["iters"] == io["iters"], w
            else:
                assert _rel(z, zo) < MIXED_PRECOND_BAR["mixed16"], w
                assert st["iters"] <= math.ceil(1.1 * io["iters"]), w
