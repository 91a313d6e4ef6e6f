"""The C-ABI library without a GPU: it loads, exports every symbol that
include/coarse.h declares, and its host-side setup (a dry run that touches no
device) builds the same subdomains and reduced space as the oracle."""
import os
import re

import numpy as np
import pytest

from oracle import fem, reduced, schwarz
from paper_2606_20496_amd import coarse, meshgen as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "coarse.h")

pytestmark = pytest.mark.skipif(not os.path.exists(coarse.LIB_PATH), reason="library not built")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(coarse_[a-z_A-Z]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    L = coarse.load()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(coarse.EXPORTS)


def test_strerror():
    L = coarse.load()
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert L.coarse_strerror(code)


def _oracle_sets(m, overlap=1):
    sets = schwarz.overlapping_subdomains(m.e2v, m.part, m.n_part, overlap)
    return schwarz.restriction_sets(m.e2v, sets, m.dirichlet)


@pytest.mark.parametrize("overlap", [1, 2])
def test_plan_matches_oracle_subdomains(overlap):
    for m in (mg.small_cube(), mg.box_mesh((9, 7, 5), 3, block=3, boxes=(3, 2, 2), faces=("z1",)),
              mg.annulus_mesh(8, 2, block=4, boxes=(2, 2, 2))):
        info, sizes = coarse.plan_info(m.xyz, m.e2v, m.dirichlet, m.part, m.n_part, overlap=overlap,
                                       boxes=m.boxes)
        R = _oracle_sets(m, overlap)
        assert sizes.tolist() == [len(r) for r in R]
        assert info["n_free"] == m.n_free
        assert info["sum_np"] == sum(len(r) for r in R)


def test_plan_matches_oracle_reduced_space():
    for m in (mg.small_cube(), mg.annulus_mesh(12, 5, block=4, boxes=(3, 3, 3)),
              mg.box_mesh(8, 4, block=4, boxes=(8, 8, 8), jitter=0.0)):
        A, Ae, Afull, free, fidx = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
        S = reduced.CentroidSpace(m.xyz, m.e2v, m.dirichlet, Ae, m.boxes, fidx, fem.multiplicity(m.e2v, m.n_vert))
        info, _ = coarse.plan_info(m.xyz, m.e2v, m.dirichlet, m.part, m.n_part, boxes=m.boxes)
        assert info["n_r"] == S.n_r
        assert info["n_cells"] == len(np.unique(S.cells[:, 0] + 1000 * S.cells[:, 1] + 10 ** 6 * S.cells[:, 2]))
        # J entries: distinct (free vertex, cell of an incident element) pairs
        cid = S.cells[:, 0] + 1000 * S.cells[:, 1] + 10 ** 6 * S.cells[:, 2]
        v = fidx[np.asarray(m.e2v)]
        pairs = np.unique(np.stack([v.ravel(), np.repeat(cid, 8)], 1)[v.ravel() >= 0], axis=0)
        assert info["n_jent"] == len(pairs)


def test_plan_partition_by_bisection():
    m = mg.box_mesh(8, 1, block=4, boxes=(2, 2, 2))
    info, sizes = coarse.plan_info(m.xyz, m.e2v, m.dirichlet, None, 8, boxes=m.boxes)
    # RCB of a cube into 8 pieces gives the 4^3 blocks again
    assert sorted(sizes.tolist()) == [100] * 4 + [125] * 4


def test_plan_rejects_bad_meshes():
    m = mg.small_cube()
    e2v = m.e2v.copy()
    e2v[3, 2] = e2v[3, 5]
    with pytest.raises(coarse.CoarseError) as ei:
        coarse.plan_info(m.xyz, e2v, m.dirichlet, m.part, m.n_part, boxes=m.boxes)
    assert ei.value.code == -3
    e2v = m.e2v.copy()
    e2v[0, 0] = m.n_vert
    with pytest.raises(coarse.CoarseError) as ei:
        coarse.plan_info(m.xyz, e2v, m.dirichlet, m.part, m.n_part, boxes=m.boxes)
    assert ei.value.code == -1
    part = m.part.copy()
    part[0] = m.n_part
    with pytest.raises(coarse.CoarseError):
        coarse.plan_info(m.xyz, m.e2v, m.dirichlet, part, m.n_part, boxes=m.boxes)


def test_solver_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    m = mg.small_cube()
    with pytest.raises(RuntimeError):
        coarse.CoarseSolver.from_mesh(m)


def test_plan_is_host_only():
    # the host half of a setup runs without any GPU (this machine may have none)
    m = mg.small_cube()
    pl = coarse.Plan.from_mesh(m, precision="mixed")
    assert pl._plan
    pl.close()
    pl.close()                      # idempotent
    with pytest.raises(coarse.CoarseError) as ei:
        coarse.Plan(m.xyz, m.e2v, m.dirichlet, m.part, m.n_part, boxes=m.boxes, max_it=0)
    assert ei.value.code == -1


def test_plan_standard_interp_matches_oracle():
    # vertex-based J (Sec. 4, eq. (Psi)): the same active box vertices as the oracle
    for m in (mg.small_cube(), mg.annulus_mesh(12, 5, block=4, boxes=(3, 3, 3))):
        A, Ae, Afull, free, fidx = fem.stiffness(m.xyz, m.e2v, m.dirichlet)
        S = reduced.StandardSpace(m.xyz, m.dirichlet, A, m.boxes, free)
        info, _ = coarse.plan_info(m.xyz, m.e2v, m.dirichlet, m.part, m.n_part, boxes=m.boxes, interp="standard")
        assert info["n_r"] == S.n_r
        assert info["n_jent"] == free.size          # one entry per free vertex


def test_plan_flags_blocks_of_mixed_element_orientation():
    # consistently oriented elements never hold one vertex at the same local
    # corner, so every operator block sums corner by corner; turning each
    # element's local numbering by a random rotation of the cube makes blocks
    # fall back to incidence lists, with the subdomains and the reduced space
    # unchanged
    m = mg.box_mesh((10, 9, 7), 21, block=4, boxes=(3, 3, 2), faces=("y1",))
    r = mg.reorient(m, 7)
    info, sizes = coarse.plan_info(m.xyz, m.e2v, m.dirichlet, m.part, m.n_part, boxes=m.boxes)
    info_r, sizes_r = coarse.plan_info(r.xyz, r.e2v, r.dirichlet, r.part, r.n_part, boxes=r.boxes)
    assert info["n_inc_blocks"] == 0
    n_blocks = -(-m.n_elem // 256)
    assert 0 < info_r["n_inc_blocks"] <= n_blocks
    assert list(sizes) == list(sizes_r)
    for k in ("n_free", "n_sub", "sum_np", "n_r", "n_cells", "n_jent"):
        assert info[k] == info_r[k], k


def test_noalloc_batch_rejects_too_many_systems():
    # the size check comes before any device call, so it runs without a GPU
    import ctypes
    L = coarse.load()
    n = coarse.NOALLOC_MAX_SOLVES + 1
    arr = (ctypes.c_void_p * n)()
    st = (coarse._Stats * n)()
    assert L.coarse_solve_batch_noalloc(arr, arr, arr, n, 1e-8, st) == -1
    assert b"COARSE_NOALLOC_MAX_SOLVES" in L.coarse_last_error(None)
    assert L.coarse_solve_batch_noalloc(arr, arr, arr, 0, 1e-8, st) == 0
