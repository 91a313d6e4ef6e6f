"""The allocation-free lock-step batch (coarse_solve_batch_noalloc) against the
allocating one (coarse_solve_batch), through the C-ABI: the same solves in the
same order of arithmetic, so every result must agree bit for bit. Two calls in a
row share the library's fixed tables; the second has fewer and smaller systems."""
import numpy as np
import pytest

from paper_2606_20496_amd import coarse, meshgen as mg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _meshes():
    out = []
    for k, (n, block, face) in enumerate(((9, 4, ("x0",)), (7, 3, ("z1",)), (11, 4, ("y0",)),
                                          (6, 3, ("x1",)), (10, 5, ("z0",)))):
        nb = -(-n // block)
        out.append(mg.box_mesh(n, 700 + k, block=block, boxes=(nb,) * 3, faces=face))
    return out


def _run(solvers, meshes, noalloc):
    bs = [torch.tensor(m.b, device="cuda") for m in meshes]
    us = [torch.full_like(b, np.nan) for b in bs]
    _, st = coarse.solve_batch(solvers, bs, tol=1e-8, outs=us, noalloc=noalloc)
    torch.cuda.synchronize()
    return [u.cpu().numpy() for u in us], st


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_batch_equals_allocating_batch(precision):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    coarse.load()
    meshes = _meshes()
    solvers = [coarse.CoarseSolver.from_mesh(m, precision=precision) for m in meshes]
    try:
        # first call: all five systems; second call: two of them, the smaller ones
        for sel in ([0, 1, 2, 3, 4], [3, 1]):
            S = [solvers[i] for i in sel]
            M = [meshes[i] for i in sel]
            ua, sa = _run(S, M, noalloc=False)
            un, sn = _run(S, M, noalloc=True)
            for k in range(len(sel)):
                assert sn[k]["status"] == 0 and sn[k]["relres"] <= 1e-8
                assert sn[k]["iters"] == sa[k]["iters"]
                assert sn[k]["relres"] == sa[k]["relres"]
                assert sn[k]["relres_true"] == sa[k]["relres_true"]
                assert np.array_equal(un[k], ua[k])
            # and each equals the solo solve of its context
            for k, i in enumerate(sel):
                u1, s1 = solvers[i].solve(torch.tensor(meshes[i].b, device="cuda"), 1e-8)
                assert s1["iters"] == sn[k]["iters"]
                assert np.array_equal(u1.cpu().numpy(), un[k])
    finally:
        for S in solvers:
            S.close()
