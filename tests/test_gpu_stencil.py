"""The reduced operator as a 27-point stencil on the structured box grid, and the
iterative refinement of the reduced solve that uses it.

* The stencil sweep w = A_r y against the oracle's cell-assembled A_r (Sec. 4,
  eq. (Aij)) at 1e-13, relative, max norm; inactive box vertices neither read
  nor written (0).
* Refinement of the reduced solve in the mixed forms: the reduced term J A_r^{-1}
  J^T r against the FP64 oracle. Without refinement its error is that of the
  stored inverse (FP32, or FP16 storage with FP32 sums); one step of refinement
  squares that and leaves the error of the FP32 interpolation and FP32
  right-hand side, bounded by 16 FP32 unit roundoffs (the bar of one mixed
  application). With FP64 inverses refinement changes nothing beyond rounding
  (1e-12)."""
import math

import numpy as np
import pytest

from oracle import problem
from paper_2606_20496_amd import coarse, meshgen as mg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24


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


MESHES = [
    ("cube8", lambda: mg.small_cube()),
    ("ragged", lambda: mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",))),
    ("annulus", lambda: mg.annulus_mesh(12, 22, block=4, boxes=(3, 3, 3))),
    ("reoriented", lambda: mg.reorient(mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",)), 7)),
    ("big_reduced", lambda: mg.box_mesh((24, 24, 20), 24, block=2, boxes=(12, 12, 10), faces=("x1",))),
    ("stretched", lambda: mg.box_mesh(16, 25, block=8, boxes=(2, 2, 2), faces=("z1",), zstretch=(1.1, 20.0))),
]


@pytest.mark.parametrize("name,make", MESHES, ids=[m[0] for m in MESHES])
def test_stencil_sweep_matches_oracle(name, make):
    m = make()
    P = problem.from_mesh(m)
    S = coarse.CoarseSolver.from_mesh(m)
    sp = P.coarse
    nbv = int(np.prod(sp.b + 1))
    assert tuple(S.info["boxes"]) == tuple(int(b) for b in sp.b) and S.info["n_r"] == sp.n_r
    rng = np.random.default_rng(61)
    for _ in range(2):
        ya = rng.standard_normal(sp.n_r)
        y = np.full(nbv, np.nan)            # inactive box vertices must not be read
        y[sp.active] = ya
        w = _np(S.apply_reduced_operator(_gpu(y)))
        ref = sp.Ar_sparse @ ya
        assert _rel(w[sp.active], ref) < 1e-13
        inactive = np.ones(nbv, bool)
        inactive[sp.active] = False
        assert np.all(w[inactive] == 0)


def test_stencil_is_27_point():
    # the structure the sweep relies on: the oracle's A_r couples box vertices at
    # most one box apart per direction
    m = mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",))
    sp = problem.from_mesh(m).coarse
    nx1, ny1 = sp.b[0] + 1, sp.b[1] + 1
    ijk = np.stack([sp.active % nx1, (sp.active // nx1) % ny1, sp.active // (nx1 * ny1)], 1)
    A = sp.Ar_sparse.tocoo()
    assert np.abs(ijk[A.row] - ijk[A.col]).max() <= 1


def _reduced_term_errors(m, precision):
    P = problem.from_mesh(m, mode="coarse_only")
    r = np.random.default_rng(62).standard_normal(m.n_vert)
    ref = P.apply_precond(r)
    out = {}
    for refine in (0, 1):
        S = coarse.CoarseSolver.from_mesh(m, mode="reduced_only", precision=precision, reduced_refine=refine)
        out[refine] = _rel(_np(S.apply_precond(_gpu(r))), ref)
    return out


@pytest.mark.parametrize("name,make", MESHES, ids=[m[0] for m in MESHES])
def test_refinement_of_the_reduced_solve(name, make):
    m = make()
    e16 = _reduced_term_errors(m, "mixed16")
    e32 = _reduced_term_errors(m, "mixed")
    e64 = _reduced_term_errors(m, "fp64")
    print(f"reduced term error {name}: mixed16 {e16}, mixed {e32}, fp64 {e64}")
    # one step squares the relative error of the FP16-stored inverse (bar 4 FP16
    # units) and adds that of the FP32 interpolation
    assert e16[1] <= (4 * 2.0 ** -11) ** 2 + 16 * U32 and e16[1] < 0.1 * e16[0]
    assert e32[1] <= 16 * U32
    assert e64[0] < 1e-12 and e64[1] < 1e-12


@pytest.fixture(scope="module")
def cube64_oracle():
    m = mg.gpu_share_cube()
    _, io = problem.from_mesh(m).solve(m.b, tol=1e-8)
    return m, io


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["mixed", "mixed16"])
def test_refined_solves(precision, cube64_oracle):
    # the whole additive preconditioner with a refined reduced solve on the 64^3
    # share: the 1e-8 residual within the mixed forms' iteration bar, and
    # repeatable bit for bit
    m, io = cube64_oracle
    S = coarse.CoarseSolver.from_mesh(m, precision=precision, reduced_refine=1)
    b = _gpu(m.b)
    u1, st = S.solve(b)
    u2, _ = S.solve(b)
    assert st["code"] == 0 and st["relres_true"] <= 1.01e-8
    assert st["iters"] <= max(math.ceil(1.1 * io["iters"]), io["iters"] + 2)
    assert torch.equal(u1, u2)


def test_refined_reduced_solve_on_the_second_stream():
    # a reduced system of 59 tile rows runs on the context's second stream; its
    # refinement goes with it
    m = MESHES[4][1]()
    S = coarse.CoarseSolver.from_mesh(m, precision="mixed16", reduced_refine=1)
    assert S.info["reduced_stream"] == 1 and S.info["reduced_refine"] == 1
    P = problem.from_mesh(m)
    r = np.random.default_rng(63).standard_normal(m.n_vert)
    ref = P.apply_precond(r)
    S0 = coarse.CoarseSolver.from_mesh(m, precision="mixed16")
    e1 = _rel(_np(S.apply_precond(_gpu(r))), ref)
    e0 = _rel(_np(S0.apply_precond(_gpu(r))), ref)
    print(f"second-stream mixed16 preconditioner error: plain {e0:.3e}, refined {e1:.3e}")
    # the local part keeps its FP16-storage error (the bar of 4 FP16 units)
    assert e1 <= 4 * 2.0 ** -11


def test_refinement_and_stencil_rejected_where_unsupported():
    m = mg.small_cube()
    with pytest.raises(coarse.CoarseError) as ei:
        coarse.CoarseSolver.from_mesh(m, interp="standard", reduced_refine=1)
    assert ei.value.code == -1
    S = coarse.CoarseSolver.from_mesh(m, interp="standard")
    nbv = int(np.prod([b + 1 for b in S.info["boxes"]]))
    with pytest.raises(coarse.CoarseError):
        S.apply_reduced_operator(_gpu(np.zeros(nbv)))
    R = coarse.CoarseSolver.from_mesh(m, precision="mixed", reduced_refine=1)
    with pytest.raises(coarse.CoarseError):
        coarse.solve_batch([R], [_gpu(m.b)])
    with pytest.raises(coarse.CoarseError):
        R.solve_multi(torch.stack([_gpu(m.b), _gpu(m.b)], 0))
