"""Seeded synthetic inputs: hexahedral meshes, boundary flags, subdomain labels and
right-hand sides for the coarse (N=1, element-vertex) Poisson problem.

This module holds no arithmetic of the solver: it only places vertices, numbers
elements and draws random numbers. Both the GPU library (through its Python
binding) and the CPU oracle consume its output, so it must stay free of anything
the method computes.

Conventions (the paper's problem statement, Sec. 3):
  * ``e2v[e, v]`` lists the 8 vertices of hexahedron ``e`` in the lexicographic
    local order ``v = i + 2 j + 4 k`` with ``(i, j, k)`` in ``{0, 1}^3``;
  * ``xyz[u]`` are vertex coordinates (float64);
  * ``dirichlet[u] = 1`` marks homogeneous Dirichlet vertices, all others are
    homogeneous Neumann;
  * ``part[e]`` is the subdomain label of element ``e`` (contiguous blocks of the
    logical grid, standing in for the paper's partitioner).

Random draws happen in one fixed order per mesh: configuration choices (where a
workload draws them), interior-vertex jitter, vertex permutation, element
permutation, then the right-hand side.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np

FACES = ("x0", "x1", "y0", "y1", "z0", "z1")


@dataclasses.dataclass
class Mesh:
    xyz: np.ndarray            # (n_vert, 3) float64
    e2v: np.ndarray            # (n_elem, 8) int32
    dirichlet: np.ndarray      # (n_vert,) uint8
    part: np.ndarray           # (n_elem,) int32
    n_part: int
    boxes: tuple               # (b_x, b_y, b_z) box counts of the reduced grid
    b: np.ndarray              # (n_vert,) float64 right-hand side (0 on Dirichlet)
    name: str = ""
    seed: int = 0
    dims: tuple = (0, 0, 0)    # logical element counts (nx, ny, nz)

    @property
    def n_vert(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_elem(self) -> int:
        return int(self.e2v.shape[0])

    @property
    def n_free(self) -> int:
        return int(self.n_vert - int(self.dirichlet.sum()))


def _logical_grid(nx: int, ny: int, nz: int):
    """Vertex ids ``i + (nx+1)(j + (ny+1) k)`` and the 8 vertex ids of every element
    in lexicographic local order; elements are numbered ``ex + nx (ey + ny ez)``."""
    sx, sy = nx + 1, (nx + 1) * (ny + 1)
    ex, ey, ez = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ex, ey, ez = ex.ravel(order="F"), ey.ravel(order="F"), ez.ravel(order="F")
    base = ex + sx * ey + sy * ez
    e2v = np.empty((base.size, 8), dtype=np.int64)
    for v in range(8):
        i, j, k = v & 1, (v >> 1) & 1, (v >> 2) & 1
        e2v[:, v] = base + i + sx * j + sy * k
    return e2v, (ex, ey, ez)


def _vertex_ijk(nx: int, ny: int, nz: int):
    i, j, k = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    return i.ravel(order="F"), j.ravel(order="F"), k.ravel(order="F")


def _block_labels(ecoords, dims, block):
    """Subdomain label of each element: logical blocks of ``block`` elements per
    axis (the last block along an axis is smaller when ``block`` does not divide
    the element count)."""
    nbx = [int(math.ceil(d / block)) for d in dims]
    bx, by, bz = (c // block for c in ecoords)
    return (bx + nbx[0] * (by + nbx[1] * bz)).astype(np.int32), int(np.prod(nbx))


def _face_mask(i, j, k, dims, face):
    nx, ny, nz = dims
    return {
        "x0": i == 0, "x1": i == nx, "y0": j == 0,
        "y1": j == ny, "z0": k == 0, "z1": k == nz,
    }[face]


def _finish(rng, xyz, e2v, dirichlet, part, n_part, boxes, permute, rhs, name, seed, dims,
            bumps=0, noise=0.0):
    n_vert, n_elem = xyz.shape[0], e2v.shape[0]
    if permute:
        vperm = rng.permutation(n_vert)          # logical vertex g -> user id vperm[g]
        eperm = rng.permutation(n_elem)          # logical element e -> user id eperm[e]
    else:
        vperm = np.arange(n_vert)
        eperm = np.arange(n_elem)
    xyz_u = np.empty_like(xyz)
    xyz_u[vperm] = xyz
    dir_u = np.empty_like(dirichlet)
    dir_u[vperm] = dirichlet
    e2v_u = np.empty_like(e2v)
    e2v_u[eperm] = vperm[e2v]
    part_u = np.empty_like(part)
    part_u[eperm] = part
    if rhs == "normal":
        b = rng.standard_normal(n_vert)
    elif rhs == "bumps":
        lo, hi = xyz_u.min(0), xyz_u.max(0)
        centres = lo + (hi - lo) * rng.random((bumps, 3))
        amps = rng.standard_normal(bumps)
        b = np.zeros(n_vert)
        for c, a in zip(centres, amps):
            b += a * np.exp(-((xyz_u - c) ** 2).sum(1) / (2.0 * 0.05 ** 2))
        b += noise * rng.standard_normal(n_vert)
    else:
        raise ValueError(rhs)
    b[dir_u.astype(bool)] = 0.0
    return Mesh(xyz=np.ascontiguousarray(xyz_u, dtype=np.float64),
                e2v=np.ascontiguousarray(e2v_u, dtype=np.int32),
                dirichlet=np.ascontiguousarray(dir_u, dtype=np.uint8),
                part=np.ascontiguousarray(part_u, dtype=np.int32), n_part=int(n_part),
                boxes=tuple(int(x) for x in boxes), b=b, name=name, seed=seed,
                dims=tuple(int(d) for d in dims))


def box_mesh(n, seed, *, block, boxes, jitter=0.1, permute=True, faces=("x0",), rhs="normal",
             bumps=20, noise=1e-3, name="", zstretch=None, rng=None):
    """Unit-cube ``n^3`` (or ``(nx,ny,nz)``) Q1 hex mesh.

    Interior vertices move by U(-jitter*h, jitter*h) per coordinate, where h is
    the local logical spacing; boundary vertices stay on the faces so that the
    union of the elements is exactly the unit cube. ``zstretch=(ratio, cap)``
    grades the z spacing geometrically (spacing of layer k proportional to
    ``min(ratio**k, cap)``), normalised to [0, 1].
    """
    dims = (n, n, n) if np.isscalar(n) else tuple(n)
    nx, ny, nz = dims
    rng = np.random.default_rng(seed) if rng is None else rng
    e2v, ecoords = _logical_grid(nx, ny, nz)
    i, j, k = _vertex_ijk(nx, ny, nz)
    # logical coordinates, jittered in index space (interior vertices only)
    jit = rng.uniform(-jitter, jitter, size=(i.size, 3))
    interior = (i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)
    li = i + np.where(interior, jit[:, 0], 0.0)
    lj = j + np.where(interior, jit[:, 1], 0.0)
    lk = k + np.where(interior, jit[:, 2], 0.0)
    xyz = np.empty((i.size, 3))
    xyz[:, 0] = li / nx
    xyz[:, 1] = lj / ny
    if zstretch is None:
        xyz[:, 2] = lk / nz
    else:
        ratio, cap = zstretch
        widths = np.minimum(ratio ** np.arange(nz), cap)
        edges = np.concatenate([[0.0], np.cumsum(widths)])
        edges /= edges[-1]
        kk = np.clip(np.floor(lk).astype(np.int64), 0, nz - 1)
        xyz[:, 2] = edges[kk] + (lk - kk) * (edges[kk + 1] - edges[kk])
    dirichlet = np.zeros(i.size, dtype=np.uint8)
    for f in faces:
        dirichlet |= _face_mask(i, j, k, dims, f).astype(np.uint8)
    part, n_part = _block_labels(ecoords, dims, block)
    return _finish(rng, xyz, e2v, dirichlet, part, n_part, boxes, permute, rhs, name, seed,
                   dims, bumps=bumps, noise=noise)


def annulus_mesh(n, seed, *, block, boxes, ratio=1.05, jitter=0.05, permute=True, name=""):
    """Quarter annulus r in [1,2], theta in [0, pi/2], z in [0,1] from an ``n^3``
    logical grid. Radial spacing grows geometrically by ``ratio`` per layer; the
    jitter is applied in index space (a fraction of the local logical spacing in
    each direction) before the mapping, so thin elements at r=1 stay valid.
    Dirichlet on r = 1, Neumann elsewhere; RHS i.i.d. N(0,1)."""
    nx = ny = nz = n
    rng = np.random.default_rng(seed)
    e2v, ecoords = _logical_grid(nx, ny, nz)
    i, j, k = _vertex_ijk(nx, ny, nz)
    jit = rng.uniform(-jitter, jitter, size=(i.size, 3))
    interior = (i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)
    li = i + np.where(interior, jit[:, 0], 0.0)
    lj = j + np.where(interior, jit[:, 1], 0.0)
    lk = k + np.where(interior, jit[:, 2], 0.0)
    # r(s) = 1 + dr0 (ratio^s - 1)/(ratio - 1), dr0 chosen so that r(n) = 2
    dr0 = (ratio - 1.0) / (ratio ** nx - 1.0)
    r = 1.0 + dr0 * (ratio ** li - 1.0) / (ratio - 1.0)
    r[i == 0] = 1.0
    r[i == nx] = 2.0
    th = 0.5 * np.pi * lj / ny
    xyz = np.empty((i.size, 3))
    xyz[:, 0] = r * np.cos(th)
    xyz[:, 1] = r * np.sin(th)
    xyz[:, 2] = lk / nz
    dirichlet = (i == 0).astype(np.uint8)
    part, n_part = _block_labels(ecoords, (nx, ny, nz), block)
    return _finish(rng, xyz, e2v, dirichlet, part, n_part, boxes, permute, "normal", name, seed,
                   (nx, ny, nz))


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def small_cube(seed=1):
    """8^3 unit cube, jitter 0.1h, Dirichlet on x=0, 8 subdomains of 4^3 elements,
    2 boxes per axis (3 reduced grid points per axis), RHS i.i.d. N(0,1)."""
    return box_mesh(8, seed, block=4, boxes=(2, 2, 2), name="cube8")


def gpu_share_cube(seed=2, n=64):
    """64^3 unit cube (one GPU's share), jitter 0.1h, Dirichlet on x=0, 512
    subdomains of 8^3 elements, 8 boxes per axis (9 grid points), RHS = 20
    Gaussian bumps of width 0.05 plus N(0, 1e-3) noise."""
    return box_mesh(n, seed, block=8, boxes=(n // 8,) * 3, rhs="bumps", name=f"cube{n}")


def large_annulus(seed=3, n=128):
    """128^3 quarter annulus, radial ratio 1.05, jitter 0.05 of the local spacing,
    4096 subdomains of 8^3 elements, 16 boxes per axis (17 grid points)."""
    return annulus_mesh(n, seed, block=8, boxes=(n // 8,) * 3, name=f"annulus{n}")


def batch_meshes(count=64, seed0=4000, nmin=6, nmax=48):
    """``count`` independent cubes, each with its own seed: n log-uniform in
    [nmin, nmax], subdomain block drawn from {4, 6, 8}, Dirichlet face drawn from
    the six faces, jitter 0.1h, boxes = ceil(n / block) per axis."""
    out = []
    for m in range(count):
        rng = np.random.default_rng(seed0 + m)
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        block = int(rng.choice([4, 6, 8]))
        face = FACES[int(rng.integers(6))]
        nb = int(math.ceil(n / block))
        out.append(box_mesh(n, seed0 + m, block=block, boxes=(nb,) * 3, faces=(face,),
                            name=f"batch{m}", rng=rng))
    return out


def serving_request_n(k, seed0=5000, nmin=8, nmax=96):
    """Edge length n of serving request ``k``'s mesh (the first draw that
    ``serving_request_mesh`` makes), without building the mesh."""
    rng = np.random.default_rng(seed0 + k)
    return int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))


def serving_request_mesh(k, seed0=5000, nmin=8, nmax=96):
    """Mesh of serving request ``k``: n log-uniform in [nmin, nmax], z spacing
    graded by 1.1 per layer with the aspect stretch capped at 20, jitter 0.1 of
    the local spacing, Dirichlet face drawn from the six faces, 8^3 subdomains
    (smaller last block), boxes = ceil(n/8) per axis."""
    rng = np.random.default_rng(seed0 + k)
    n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    face = FACES[int(rng.integers(6))]
    nb = int(math.ceil(n / 8))
    return box_mesh(n, seed0 + k, block=8, boxes=(nb,) * 3, faces=(face,),
                    zstretch=(1.1, 20.0), name=f"req{k}", rng=rng)


def serving_arrivals(rate, count=4096, seed=59999, reuse=0.3):
    """Poisson arrival times at ``rate`` requests/s and, per request, the mesh id
    it uses (a fresh one, or with probability ``reuse`` an earlier one) and the
    seed of its RHS."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    mesh_id = np.empty(count, dtype=np.int64)
    fresh = 0
    for q in range(count):
        if q > 0 and rng.random() < reuse:
            mesh_id[q] = mesh_id[int(rng.integers(q))]
        else:
            mesh_id[q] = fresh
            fresh += 1
    rhs_seed = rng.integers(0, 2 ** 31 - 1, size=count)
    return t, mesh_id, rhs_seed


def _cube_rotations():
    """The 24 proper rotations of the reference cube as maps of local vertex
    v = i + 2j + 4k: (axis permutation, flips) with determinant +1, each given
    as the array new_local[v]."""
    out = []
    for perm in itertools.permutations(range(3)):
        inversions = sum(1 for a in range(3) for b in range(a + 1, 3) if perm[a] > perm[b])
        for flips in itertools.product((0, 1), repeat=3):
            if (inversions + sum(flips)) % 2:
                continue
            m = np.empty(8, dtype=np.int64)
            for v in range(8):
                c = (v & 1, (v >> 1) & 1, (v >> 2) & 1)
                cn = [c[perm[d]] ^ flips[d] for d in range(3)]
                m[v] = cn[0] + 2 * cn[1] + 4 * cn[2]
            out.append(m)
    return out


def reorient(mesh: Mesh, seed: int) -> Mesh:
    """The same mesh with each element's local vertex numbering turned by one of
    the 24 rotations of the reference cube (drawn per element from ``seed``):
    the elements, and so the operator, are unchanged, but neighbouring elements
    no longer hold a shared vertex at matching local corners, as in meshes from
    an unstructured mesher."""
    rots = _cube_rotations()
    pick = np.random.default_rng(seed).integers(0, len(rots), size=mesh.n_elem)
    e2v = np.empty_like(mesh.e2v)
    for r, m in enumerate(rots):
        sel = pick == r
        e2v[np.ix_(sel, m)] = mesh.e2v[sel]
    return dataclasses.replace(mesh, e2v=np.ascontiguousarray(e2v), name=mesh.name + "_reoriented")


def resident_arrivals(rate, count, n_keys, seed=58999):
    """Poisson arrival times at ``rate`` requests/s over ``n_keys`` meshes that are
    all resident: per request, its mesh drawn uniformly and the seed of its RHS."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    key = rng.integers(0, n_keys, size=count)
    rhs_seed = rng.integers(0, 2 ** 31 - 1, size=count)
    return t, key, rhs_seed


def rhs_bumps(mesh: Mesh, seed: int, bumps: int = 20, noise: float = 1e-3) -> np.ndarray:
    """A fresh RHS of ``bumps`` Gaussian bumps (width 0.05, centres uniform in the
    bounding box, amplitudes N(0,1)) plus N(0, noise^2) values (0 on Dirichlet)."""
    rng = np.random.default_rng(seed)
    lo, hi = mesh.xyz.min(0), mesh.xyz.max(0)
    centres = lo + (hi - lo) * rng.random((bumps, 3))
    amps = rng.standard_normal(bumps)
    b = np.zeros(mesh.n_vert)
    for c, a in zip(centres, amps):
        b += a * np.exp(-((mesh.xyz - c) ** 2).sum(1) / (2.0 * 0.05 ** 2))
    b += noise * rng.standard_normal(mesh.n_vert)
    b[mesh.dirichlet.astype(bool)] = 0.0
    return b


def rhs_sequence(mesh: Mesh, seed: int, steps: int, dt: float = 0.005, bumps: int = 20,
                 noise: float = 0.0) -> list:
    """Right-hand sides at ``steps`` successive times t_m = m dt of a load that
    changes smoothly in time, as a pressure equation sees it step after step:
    ``bumps`` Gaussian bumps (width 0.05) whose centres start uniform in the
    bounding box and move with fixed N(0, 1) velocities (in units of the box size
    per unit time), with amplitudes a_k cos(w_k t + phi_k), a_k ~ N(0, 1),
    w_k uniform in [1, 4], phi_k uniform in [0, 2 pi); plus fresh N(0, noise^2)
    values at each step. Dirichlet entries 0."""
    rng = np.random.default_rng(seed)
    lo, hi = mesh.xyz.min(0), mesh.xyz.max(0)
    c0 = lo + (hi - lo) * rng.random((bumps, 3))
    vel = (hi - lo) * rng.standard_normal((bumps, 3))
    amp = rng.standard_normal(bumps)
    omega = rng.uniform(1.0, 4.0, bumps)
    phase = rng.uniform(0.0, 2.0 * np.pi, bumps)
    dmask = mesh.dirichlet.astype(bool)
    out = []
    for m in range(steps):
        t = m * dt
        b = np.zeros(mesh.n_vert)
        for k in range(bumps):
            c = c0[k] + vel[k] * t
            b += amp[k] * np.cos(omega[k] * t + phase[k]) * np.exp(-((mesh.xyz - c) ** 2).sum(1) / (2.0 * 0.05 ** 2))
        if noise > 0.0:
            b += noise * rng.standard_normal(mesh.n_vert)
        b[dmask] = 0.0
        out.append(b)
    return out


def rhs_normal(mesh: Mesh, seed: int) -> np.ndarray:
    """A fresh i.i.d. N(0,1) RHS for ``mesh`` (0 on Dirichlet vertices)."""
    b = np.random.default_rng(seed).standard_normal(mesh.n_vert)
    b[mesh.dirichlet.astype(bool)] = 0.0
    return b


WORKLOADS = {
    "cube8": small_cube,
    "cube64": gpu_share_cube,
    "annulus128": large_annulus,
}
