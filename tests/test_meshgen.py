"""The seeded input generator: reproducible, the sizes of the five workloads,
valid (positively oriented) elements, boundary vertices left on the faces, and
numberings that are bijections."""
import numpy as np

from paper_2606_20496_amd import meshgen as mg


def _signed_volumes(m):
    X = m.xyz[m.e2v]
    # one tetrahedron at vertex 0 spanned by the three edge neighbours 1, 2, 4
    a, b, c = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 4] - X[:, 0]
    return np.einsum("ei,ei->e", a, np.cross(b, c))


def test_reproducible():
    a, b = mg.small_cube(), mg.small_cube()
    for f in ("xyz", "e2v", "dirichlet", "part", "b"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = mg.small_cube(seed=9)
    assert not np.array_equal(a.xyz, c.xyz)


def test_small_cube_shape():
    m = mg.small_cube()
    assert (m.n_vert, m.n_elem, m.n_free, m.n_part, m.boxes) == (729, 512, 648, 8, (2, 2, 2))
    assert np.all(np.bincount(m.part) == 64)
    assert sorted(np.unique(m.e2v)) == list(range(729))
    assert np.all(m.b[m.dirichlet.astype(bool)] == 0)
    assert _signed_volumes(m).min() > 0
    # boundary vertices on the faces, Dirichlet exactly on x = 0
    on_face = np.any((m.xyz == 0) | (m.xyz == 1), axis=1)
    assert on_face.sum() == 729 - 7 ** 3
    assert np.all(m.xyz[m.dirichlet.astype(bool), 0] == 0)


def test_annulus_shape():
    m = mg.annulus_mesh(8, 3, block=4, boxes=(2, 2, 2))
    r = np.hypot(m.xyz[:, 0], m.xyz[:, 1])
    assert abs(r.min() - 1) < 1e-15 and abs(r.max() - 2) < 1e-15
    assert np.allclose(r[m.dirichlet.astype(bool)], 1.0)
    assert _signed_volumes(m).min() > 0


def test_batch_and_serving_draws():
    ms = mg.batch_meshes(count=6)
    for m in ms:
        assert 6 <= m.dims[0] <= 48 and m.dirichlet.sum() > 0
        assert _signed_volumes(m).min() > 0
    m = mg.serving_request_mesh(3)
    dz = np.diff(np.unique(np.round(m.xyz[:, 2], 12)))
    assert _signed_volumes(m).min() > 0 and m.n_part >= 1
    t, ids, seeds = mg.serving_arrivals(100.0, count=500)
    assert np.all(np.diff(t) > 0) and ids.max() < 500
    reuse = np.mean([ids[q] in ids[:q] for q in range(1, 500)])
    assert 0.2 < reuse < 0.4


def test_reorient_keeps_the_operator():
    # 24 distinct proper rotations; the assembled operator is the same matrix
    from oracle import fem
    rots = mg._cube_rotations()
    assert len({tuple(r) for r in rots}) == 24
    m = mg.small_cube()
    r = mg.reorient(m, 5)
    assert not np.array_equal(r.e2v, m.e2v)
    assert np.array_equal(np.sort(r.e2v, axis=1), np.sort(m.e2v, axis=1))
    d = m.dirichlet.astype(bool)
    A1 = fem.stiffness(m.xyz, m.e2v, d)[0]
    A2 = fem.stiffness(r.xyz, r.e2v, d)[0]
    assert abs(A1 - A2).max() <= 1e-14 * abs(A1).max()
