"""The knife-edge iteration bar (oracle only, CPU): on a batch-workload mesh
whose residual crosses 1e-8 within rounding at iteration 21 (9.78e-9 there),
the oracle itself stops at 21 or 22 under 1e-13 perturbations of b or of its
preconditioner's output, so both counts are accepted; on the small cube the
count does not move, and a count one off is rejected."""
import pytest

from iteration_bar import check_fp64_iters, oracle_counts
from oracle import problem
from paper_2606_20496_amd import meshgen as mg


def test_knife_edge_mesh_admits_both_counts():
    m = mg.batch_meshes(count=64)[20]
    P = problem.from_mesh(m)
    _, io = P.solve(m.b, tol=1e-8, record=True)
    assert io["iters"] == 21 and 0.9e-8 < io["relres_hist"][-1] < 1e-8
    counts = oracle_counts(P, m.b, io["iters"])
    assert counts == {21, 22}
    check_fp64_iters(22, P, m.b, io["iters"])


def test_settled_mesh_admits_one_count():
    m = mg.small_cube()
    P = problem.from_mesh(m)
    _, io = P.solve(m.b, tol=1e-8)
    assert oracle_counts(P, m.b, io["iters"]) == {io["iters"]}
    with pytest.raises(AssertionError):
        check_fp64_iters(io["iters"] + 1, P, m.b, io["iters"])
