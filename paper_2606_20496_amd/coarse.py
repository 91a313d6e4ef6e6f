"""Python binding of ``libcoarse.so`` (the C-ABI in include/coarse.h).

Argument marshalling only: every step of setup, preconditioning and PCG runs in
the library's HIP kernels. torch provides device memory and the current stream.
There is no CPU fallback: without the built library, or without a GPU, the
calls that compute raise.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcoarse.so")

PRECISION = {"fp64": 0, "mixed": 1, "mixed16": 2}
PROJECTION_MAX = 64   # COARSE_PROJECTION_MAX: largest basis of prior solutions
MULTI_MAX = 16        # COARSE_MULTI_MAX: right-hand sides of one block solve
MODE = {"additive": 0, "hybrid_sym": 1, "local_only": 2, "reduced_only": 3, "hybrid": 4}
INTERP = {"centroid": 0, "standard": 1}
STATUS = {0: "ok", 1: "notconv", -1: "einval", -2: "enomem", -3: "emesh", -4: "esingular",
          -5: "edevice", -6: "ebreakdown"}

# every symbol declared in include/coarse.h
EXPORTS = ("coarse_default_opts", "coarse_setup", "coarse_apply_precond", "coarse_apply_A",
           "coarse_solve", "coarse_solve_batch", "coarse_destroy", "coarse_device_bytes",
           "coarse_get_info", "coarse_set_stream", "coarse_plan_info", "coarse_strerror",
           "coarse_last_error", "coarse_profile", "coarse_batch_create", "coarse_batch_submit",
           "coarse_batch_step", "coarse_batch_launch", "coarse_batch_collect", "coarse_batch_live", "coarse_batch_destroy", "coarse_plan_create",
           "coarse_setup_from_plan", "coarse_plan_destroy", "coarse_plan_set_gemv_tiles",
           "coarse_solve_projected", "coarse_projection_reset", "coarse_solve_multi",
           "coarse_apply_precond_multi", "coarse_multi_begin", "coarse_multi_advance", "coarse_multi_done",
           "coarse_multi_end", "coarse_solve_batch_noalloc", "coarse_apply_reduced_operator")
NOALLOC_MAX_SOLVES = 256   # COARSE_NOALLOC_MAX_SOLVES

PHASES = ("A+p", "R_p+J^T", "J^T corners", "A_p^-1/A_r^-1 gemv", "combine", "sum+J", "x,r update",
          "reduced branch (second stream)")


class CoarseError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class _Mesh(ctypes.Structure):
    _fields_ = [("n_vert", ctypes.c_int64), ("n_elem", ctypes.c_int64),
                ("xyz", ctypes.POINTER(ctypes.c_double)), ("e2v", ctypes.POINTER(ctypes.c_int32)),
                ("part", ctypes.POINTER(ctypes.c_int32)), ("n_part", ctypes.c_int32)]


class _BC(ctypes.Structure):
    _fields_ = [("dirichlet", ctypes.POINTER(ctypes.c_uint8))]


# Size buckets of the GEMV work-item table (upper bounds on a system's tile
# count nb = ceil(n/32), the last open), as in coarse.h.
GEMV_BUCKETS = 8
GEMV_BUCKET_MAX = (2, 4, 8, 12, 16, 24, 48, 1 << 30)
TUNING_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gemv_tuning.json")


def gemv_table(precision="fp64"):
    """Tiles per GEMV work item per size bucket for a precision: the table written
    by the tuner (``python -m paper_2606_20496_amd.tune``) if one is present, else
    4 everywhere."""
    try:
        with open(TUNING_PATH) as f:
            t = json.load(f)[precision]["tiles_per_item"]
        if len(t) == GEMV_BUCKETS and all(int(x) >= 1 for x in t):
            return [int(x) for x in t]
    except (OSError, ValueError, KeyError, TypeError):
        pass
    return [4] * GEMV_BUCKETS


def whole_waves_choice(precision="fp64"):
    """Wavefronts per whole-system workgroup for a precision from the tuner's
    table (0, the library's default, when there is none)."""
    try:
        with open(TUNING_PATH) as f:
            w = int(json.load(f)[precision].get("whole_waves", 0))
        return w if w in (0, 2, 4, 8, 16) else 0
    except (OSError, ValueError, KeyError, TypeError, AttributeError):
        return 0


class _Opts(ctypes.Structure):
    _fields_ = [("overlap", ctypes.c_int), ("boxes", ctypes.c_int * 3), ("precision", ctypes.c_int),
                ("mode", ctypes.c_int), ("interp", ctypes.c_int), ("max_it", ctypes.c_int),
                ("check_every", ctypes.c_int), ("flexible", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("gemv_tiles", ctypes.c_int * GEMV_BUCKETS), ("projection", ctypes.c_int),
                ("whole_waves", ctypes.c_int), ("block_rhs", ctypes.c_int), ("local_iters", ctypes.c_int),
                ("reduced_refine", ctypes.c_int)]


class _Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("relres", ctypes.c_double),
                ("relres_true", ctypes.c_double), ("t_setup", ctypes.c_double), ("t_solve", ctypes.c_double),
                ("relres0", ctypes.c_double), ("n_basis", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("n_free", ctypes.c_int64), ("n_sub", ctypes.c_int64), ("sum_np", ctypes.c_int64),
                ("max_np", ctypes.c_int64), ("n_r", ctypes.c_int64), ("n_cells", ctypes.c_int64),
                ("local_bytes", ctypes.c_int64), ("reduced_bytes", ctypes.c_int64),
                ("a_bytes", ctypes.c_int64), ("inv_alg_bytes", ctypes.c_int64),
                ("n_jent", ctypes.c_int64), ("n_inc_blocks", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("boxes", ctypes.c_int32 * 3), ("precision", ctypes.c_int32),
                ("gemv_tiles", ctypes.c_int32 * GEMV_BUCKETS), ("whole_waves", ctypes.c_int32),
                ("reduced_stream", ctypes.c_int32), ("local_iters", ctypes.c_int32),
                ("ell_width", ctypes.c_int32), ("reduced_refine", ctypes.c_int32)]


_lib = None


def load():
    """Load the shared library (after torch, so both use one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2606_20496_amd.build.build()")
    try:
        import torch  # noqa: F401  (loads the HIP runtime first)
    except Exception:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    L.coarse_default_opts.argtypes = [ctypes.POINTER(_Opts)]
    L.coarse_default_opts.restype = None
    L.coarse_setup.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_BC), ctypes.POINTER(_Opts),
                               ctypes.POINTER(vp)]
    L.coarse_setup.restype = i32
    L.coarse_apply_precond.argtypes = [vp, vp, vp]
    L.coarse_apply_precond.restype = i32
    L.coarse_apply_A.argtypes = [vp, vp, vp]
    L.coarse_apply_A.restype = i32
    L.coarse_apply_reduced_operator.argtypes = [vp, vp, vp]
    L.coarse_apply_reduced_operator.restype = i32
    L.coarse_solve.argtypes = [vp, vp, vp, dbl, ctypes.POINTER(_Stats)]
    L.coarse_solve.restype = i32
    L.coarse_solve_projected.argtypes = [vp, vp, vp, dbl, ctypes.POINTER(_Stats)]
    L.coarse_solve_projected.restype = i32
    L.coarse_projection_reset.argtypes = [vp]
    L.coarse_projection_reset.restype = i32
    L.coarse_solve_multi.argtypes = [vp, i32, vp, vp, dbl, ctypes.POINTER(_Stats)]
    L.coarse_solve_multi.restype = i32
    L.coarse_apply_precond_multi.argtypes = [vp, i32, vp, vp]
    L.coarse_apply_precond_multi.restype = i32
    L.coarse_multi_begin.argtypes = [vp, i32, vp, dbl]
    L.coarse_multi_begin.restype = i32
    L.coarse_multi_advance.argtypes = [vp, i32]
    L.coarse_multi_advance.restype = i32
    L.coarse_multi_done.argtypes = [vp]
    L.coarse_multi_done.restype = i32
    L.coarse_multi_end.argtypes = [vp, vp, ctypes.POINTER(_Stats)]
    L.coarse_multi_end.restype = i32
    L.coarse_solve_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i32, dbl,
                                     ctypes.POINTER(_Stats)]
    L.coarse_solve_batch.restype = i32
    L.coarse_solve_batch_noalloc.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i32, dbl,
                                             ctypes.POINTER(_Stats)]
    L.coarse_solve_batch_noalloc.restype = i32
    L.coarse_destroy.argtypes = [vp]
    L.coarse_destroy.restype = i32
    L.coarse_device_bytes.argtypes = [vp]
    L.coarse_device_bytes.restype = ctypes.c_size_t
    L.coarse_get_info.argtypes = [vp, ctypes.POINTER(_Info)]
    L.coarse_get_info.restype = i32
    L.coarse_set_stream.argtypes = [vp, vp]
    L.coarse_set_stream.restype = i32
    L.coarse_plan_info.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_BC), ctypes.POINTER(_Opts),
                                   ctypes.POINTER(_Info), ctypes.POINTER(i64)]
    L.coarse_plan_info.restype = i32
    L.coarse_strerror.argtypes = [i32]
    L.coarse_strerror.restype = ctypes.c_char_p
    L.coarse_profile.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64), i32]
    L.coarse_profile.restype = i32
    L.coarse_batch_create.argtypes = [vp, i32, ctypes.POINTER(vp)]
    L.coarse_batch_create.restype = i32
    L.coarse_batch_submit.argtypes = [vp, vp, vp, vp, dbl, i64]
    L.coarse_batch_submit.restype = i32
    L.coarse_batch_step.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(_Stats), i32, ctypes.POINTER(i32)]
    L.coarse_batch_step.restype = i32
    L.coarse_batch_launch.argtypes = [vp, i32]
    L.coarse_batch_launch.restype = i32
    L.coarse_batch_collect.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(_Stats), i32, ctypes.POINTER(i32)]
    L.coarse_batch_collect.restype = i32
    L.coarse_batch_live.argtypes = [vp]
    L.coarse_batch_live.restype = i32
    L.coarse_batch_destroy.argtypes = [vp]
    L.coarse_batch_destroy.restype = i32
    L.coarse_plan_create.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_BC), ctypes.POINTER(_Opts),
                                     ctypes.POINTER(vp)]
    L.coarse_plan_create.restype = i32
    L.coarse_setup_from_plan.argtypes = [vp, vp, ctypes.POINTER(vp)]
    L.coarse_setup_from_plan.restype = i32
    L.coarse_plan_set_gemv_tiles.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    L.coarse_plan_set_gemv_tiles.restype = i32
    L.coarse_plan_destroy.argtypes = [vp]
    L.coarse_plan_destroy.restype = i32
    L.coarse_last_error.argtypes = [vp]
    L.coarse_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _arrays(xyz, e2v, dirichlet, part, n_part):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    e2v = np.ascontiguousarray(e2v, dtype=np.int32)
    dirichlet = np.ascontiguousarray(dirichlet, dtype=np.uint8)
    if part is not None:
        part = np.ascontiguousarray(part, dtype=np.int32)
    m = _Mesh(xyz.shape[0], e2v.shape[0], xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
              e2v.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
              part.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if part is not None else None, int(n_part))
    bc = _BC(dirichlet.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return m, bc, (xyz, e2v, dirichlet, part)


def _opts(overlap, boxes, precision, mode, interp, max_it, check_every, flexible, stream, gemv_tiles=None,
          projection=0, block_rhs=0, whole_waves=None, local_iters=0, reduced_refine=0):
    o = _Opts()
    load().coarse_default_opts(ctypes.byref(o))
    o.overlap = int(overlap)
    for d in range(3):
        o.boxes[d] = int(boxes[d]) if boxes is not None else 0
    o.precision = PRECISION[precision]
    o.mode = MODE[mode]
    o.interp = INTERP[interp]
    o.max_it = int(max_it)
    o.check_every = int(check_every)
    if flexible is None:
        flexible = precision in ("mixed", "mixed16") or mode == "hybrid" or local_iters > 0
    o.flexible = int(bool(flexible))
    o.stream = stream
    t = gemv_table(precision) if gemv_tiles is None else list(gemv_tiles)
    if len(t) != GEMV_BUCKETS:
        raise ValueError(f"gemv_tiles needs {GEMV_BUCKETS} entries")
    for b in range(GEMV_BUCKETS):
        o.gemv_tiles[b] = int(t[b])
    o.projection = int(projection)
    o.block_rhs = int(bool(block_rhs))
    o.whole_waves = whole_waves_choice(precision) if whole_waves is None else int(whole_waves)
    o.local_iters = int(local_iters)
    o.reduced_refine = int(bool(reduced_refine))
    return o


def _info_dict(info):
    d = {f: getattr(info, f) for f, _ in _Info._fields_ if f not in ("boxes", "gemv_tiles")}
    d["boxes"] = tuple(info.boxes)
    d["gemv_tiles"] = tuple(info.gemv_tiles)
    return d


def plan_info(xyz, e2v, dirichlet, part=None, n_part=1, *, overlap=1, boxes=None, interp="centroid"):
    """Host-only dry run of the setup: sizes and |R_p| per subdomain (no GPU)."""
    L = load()
    m, bc, keep = _arrays(xyz, e2v, dirichlet, part, n_part)
    o = _opts(overlap, boxes, "fp64", "additive", interp, 1000, 4, False, None)
    info = _Info()
    sizes = np.zeros(max(1, int(n_part)), dtype=np.int64)
    rc = L.coarse_plan_info(ctypes.byref(m), ctypes.byref(bc), ctypes.byref(o), ctypes.byref(info),
                            sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise CoarseError(rc, L.coarse_last_error(None).decode())
    return _info_dict(info), sizes


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """The host half of a setup (coarse_plan_create): no GPU call, so it may be
    built on a worker thread while the GPU serves other solves. Takes the same
    arguments as :class:`CoarseSolver`; :meth:`CoarseSolver.from_plan` does the
    device half."""

    def __init__(self, xyz, e2v, dirichlet, part=None, n_part=1, *, overlap=1, boxes=None,
                 precision="fp64", mode="additive", interp="centroid", max_it=1000, check_every=4,
                 flexible=None, gemv_tiles=None, projection=0, block_rhs=0, whole_waves=None, local_iters=0,
                 reduced_refine=0):
        L = load()
        self._L = L
        self.n_vert = int(np.asarray(xyz).shape[0])
        self.precision = precision
        m, bc, keep = _arrays(xyz, e2v, dirichlet, part, n_part)
        o = _opts(overlap, boxes, precision, mode, interp, max_it, check_every, flexible, None, gemv_tiles,
                  projection, block_rhs, whole_waves, local_iters, reduced_refine)
        pl = ctypes.c_void_p()
        rc = L.coarse_plan_create(ctypes.byref(m), ctypes.byref(bc), ctypes.byref(o), ctypes.byref(pl))
        if rc != 0:
            raise CoarseError(rc, L.coarse_last_error(None).decode())
        self._plan = pl

    @classmethod
    def from_mesh(cls, mesh, **kw):
        kw.setdefault("boxes", mesh.boxes)
        return cls(mesh.xyz, mesh.e2v, mesh.dirichlet, mesh.part, mesh.n_part, **kw)

    def set_gemv_tiles(self, tiles):
        """Work-item table (tiles per item, per size bucket) for later device setups."""
        arr = (ctypes.c_int * GEMV_BUCKETS)(*[int(t) for t in tiles])
        rc = self._L.coarse_plan_set_gemv_tiles(self._plan, arr)
        if rc != 0:
            raise CoarseError(rc, "bad work-item table")

    def close(self):
        if getattr(self, "_plan", None):
            self._L.coarse_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CoarseSolver:
    """One mesh's two-level Schwarz PCG solver on the current GPU.

    Vectors are float64 CUDA (HIP) tensors of length ``n_vert`` in the caller's
    vertex numbering; Dirichlet entries are ignored on input and zero on output.
    """

    def __init__(self, xyz, e2v, dirichlet, part=None, n_part=1, *, overlap=1, boxes=None,
                 precision="fp64", mode="additive", interp="centroid", max_it=1000, check_every=4,
                 flexible=None, gemv_tiles=None, projection=0, block_rhs=0, whole_waves=None, local_iters=0,
                 reduced_refine=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("CoarseSolver needs a GPU; no CPU fallback exists")
        L = load()
        self._L = L
        self.n_vert = int(np.asarray(xyz).shape[0])
        self.precision = precision
        m, bc, keep = _arrays(xyz, e2v, dirichlet, part, n_part)
        o = _opts(overlap, boxes, precision, mode, interp, max_it, check_every, flexible, _stream(), gemv_tiles,
                  projection, block_rhs, whole_waves, local_iters, reduced_refine)
        ctx = ctypes.c_void_p()
        rc = L.coarse_setup(ctypes.byref(m), ctypes.byref(bc), ctypes.byref(o), ctypes.byref(ctx))
        if rc != 0:
            raise CoarseError(rc, L.coarse_last_error(None).decode())
        self._ctx = ctx
        info = _Info()
        L.coarse_get_info(ctx, ctypes.byref(info))
        self.info = _info_dict(info)

    @classmethod
    def from_mesh(cls, mesh, **kw):
        kw.setdefault("boxes", mesh.boxes)
        return cls(mesh.xyz, mesh.e2v, mesh.dirichlet, mesh.part, mesh.n_part, **kw)

    @classmethod
    def from_plan(cls, plan):
        """The device half of a setup from a :class:`Plan`, on the current stream."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("CoarseSolver needs a GPU; no CPU fallback exists")
        L = load()
        self = cls.__new__(cls)
        self._L = L
        self.n_vert = plan.n_vert
        self.precision = plan.precision
        ctx = ctypes.c_void_p()
        rc = L.coarse_setup_from_plan(plan._plan, _stream(), ctypes.byref(ctx))
        if rc != 0:
            raise CoarseError(rc, L.coarse_last_error(None).decode())
        self._ctx = ctx
        info = _Info()
        L.coarse_get_info(ctx, ctypes.byref(info))
        self.info = _info_dict(info)
        return self

    def _check(self, rc):
        if rc < 0:
            raise CoarseError(rc, self._L.coarse_last_error(self._ctx).decode())
        return rc

    def _vec(self, v):
        import torch
        if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.float64 and v.is_contiguous()
                and v.numel() == self.n_vert):
            raise ValueError("expected a contiguous float64 GPU tensor of length n_vert")
        return ctypes.c_void_p(v.data_ptr())

    def _sync_stream(self):
        self._L.coarse_set_stream(self._ctx, _stream())

    def apply_precond(self, r, out=None):
        import torch
        self._sync_stream()
        out = torch.empty_like(r) if out is None else out
        self._check(self._L.coarse_apply_precond(self._ctx, self._vec(r), self._vec(out)))
        return out

    def apply_A(self, p, out=None):
        import torch
        self._sync_stream()
        out = torch.empty_like(p) if out is None else out
        self._check(self._L.coarse_apply_A(self._ctx, self._vec(p), self._vec(out)))
        return out

    def apply_reduced_operator(self, y, out=None):
        """w = A_r y by the 27-point stencil on the box grid: y and w are float64
        GPU tensors of (b_x+1)(b_y+1)(b_z+1) entries, box vertex (i, j, k) at
        i + (b_x+1)(j + (b_y+1)k); w is 0 at inactive box vertices."""
        import torch
        self._sync_stream()
        nbv = int(np.prod([b + 1 for b in self.info["boxes"]]))
        if not (isinstance(y, torch.Tensor) and y.is_cuda and y.dtype == torch.float64 and y.is_contiguous()
                and y.numel() == nbv):
            raise ValueError(f"expected a contiguous float64 GPU tensor of {nbv} box-vertex values")
        out = torch.empty_like(y) if out is None else out
        self._check(self._L.coarse_apply_reduced_operator(self._ctx, ctypes.c_void_p(y.data_ptr()),
                                                          ctypes.c_void_p(out.data_ptr())))
        return out

    def _solve(self, fn, b, tol, out):
        import torch
        self._sync_stream()
        out = torch.empty_like(b) if out is None else out
        st = _Stats()
        rc = self._check(fn(self._ctx, self._vec(b), self._vec(out), float(tol), ctypes.byref(st)))
        stats = {f: getattr(st, f) for f, _ in _Stats._fields_}
        stats["code"] = rc
        return out, stats

    def solve(self, b, tol=1e-8, out=None):
        return self._solve(self._L.coarse_solve, b, tol, out)

    def solve_projected(self, b, tol=1e-8, out=None):
        """One solve of a sequence with the same A: PCG from the A-orthogonal
        projection onto the stored prior solutions, which then take in this one
        (needs ``projection`` >= 1 at construction)."""
        return self._solve(self._L.coarse_solve_projected, b, tol, out)

    def _block(self, v):
        import torch
        if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.float64 and v.is_contiguous()
                and v.dim() == 2 and v.shape[1] == self.n_vert and 1 <= v.shape[0] <= MULTI_MAX):
            raise ValueError(f"expected a contiguous float64 GPU tensor [k, n_vert], 1 <= k <= {MULTI_MAX}")
        return ctypes.c_void_p(v.data_ptr())

    def solve_multi(self, B, tol=1e-8, out=None):
        """Block solve of the k = B.shape[0] right-hand sides (rows of B): k PCG
        recurrences that share every read of the operator and of the stored
        inverses (additive mode, any precision). Returns (U, [stats per column])."""
        import torch
        self._sync_stream()
        out = torch.empty_like(B) if out is None else out
        k = int(B.shape[0]) if B.dim() == 2 else 0
        st = (_Stats * max(k, 1))()
        pb, pu = self._block(B), self._block(out)
        if out.shape != B.shape or out.data_ptr() == B.data_ptr():
            raise ValueError("out must be a distinct tensor of the shape of B")
        rc = self._check(self._L.coarse_solve_multi(self._ctx, k, pb, pu, float(tol), st))
        stats = []
        for j in range(k):
            d = {f: getattr(st[j], f) for f, _ in _Stats._fields_}
            d["code"] = rc
            stats.append(d)
        return out, stats

    def multi_begin(self, B, tol=1e-8):
        """Start a block solve of the rows of B without waiting for it (the
        stepped form of solve_multi); B must stay alive until multi_end."""
        self._sync_stream()
        self._check(self._L.coarse_multi_begin(self._ctx, int(B.shape[0]), self._block(B), float(tol)))
        self._multi_b = B

    def multi_advance(self, iters):
        """Enqueue `iters` iterations of the live columns (no wait)."""
        self._sync_stream()
        self._check(self._L.coarse_multi_advance(self._ctx, int(iters)))

    def multi_done(self):
        """Whether every column had finished at the last advance (call after the
        stream has been synchronised)."""
        return self._check(self._L.coarse_multi_done(self._ctx)) == 1

    def multi_end(self, out=None):
        """Finish the block solve begun by multi_begin: (U, [stats per column])."""
        import torch
        self._sync_stream()
        B = self._multi_b
        out = torch.empty_like(B) if out is None else out
        k = int(B.shape[0])
        st = (_Stats * k)()
        rc = self._check(self._L.coarse_multi_end(self._ctx, self._block(out), st))
        self._multi_b = None
        stats = []
        for j in range(k):
            d = {f: getattr(st[j], f) for f, _ in _Stats._fields_}
            d["code"] = rc
            stats.append(d)
        return out, stats

    def apply_precond_multi(self, R, out=None):
        """z_j = M r_j for the rows of R (the block form of apply_precond)."""
        import torch
        self._sync_stream()
        out = torch.empty_like(R) if out is None else out
        pr, pz = self._block(R), self._block(out)
        if out.shape != R.shape or out.data_ptr() == R.data_ptr():
            raise ValueError("out must be a distinct tensor of the shape of R")
        self._check(self._L.coarse_apply_precond_multi(self._ctx, int(R.shape[0]), pr, pz))
        return out

    def projection_reset(self):
        self._check(self._L.coarse_projection_reset(self._ctx))

    def profile_start(self, mask=0xFF):
        """Time the phases whose bits are set in ``mask`` (bit i = PHASES[i])."""
        self._check(self._L.coarse_profile(self._ctx, int(mask), None, None, 0))

    def profile_stop(self):
        """Stop the phase timers; returns {phase: (total_ms, launches)}."""
        ms = (ctypes.c_double * len(PHASES))()
        cnt = (ctypes.c_int64 * len(PHASES))()
        self._check(self._L.coarse_profile(self._ctx, 0, ms, cnt, len(PHASES)))
        return {ph: (ms[i], cnt[i]) for i, ph in enumerate(PHASES)}

    @property
    def device_bytes(self):
        return int(self._L.coarse_device_bytes(self._ctx))

    def close(self):
        if getattr(self, "_ctx", None):
            self._L.coarse_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(solvers, bs, tol=1e-8, outs=None, noalloc=False):
    """Solve several systems in lock step (one stream, shared local-solve launch).
    ``noalloc``: the allocation-free entry point (coarse_solve_batch_noalloc; at
    most NOALLOC_MAX_SOLVES systems, calls must not overlap)."""
    import torch
    L = load()
    n = len(solvers)
    outs = [torch.empty_like(b) for b in bs] if outs is None else outs
    for s in solvers:
        s._sync_stream()
    ctxs = (ctypes.c_void_p * n)(*[s._ctx.value for s in solvers])
    bp = (ctypes.c_void_p * n)(*[s._vec(b).value for s, b in zip(solvers, bs)])
    up = (ctypes.c_void_p * n)(*[s._vec(u).value for s, u in zip(solvers, outs)])
    st = (_Stats * n)()
    fn = L.coarse_solve_batch_noalloc if noalloc else L.coarse_solve_batch
    rc = fn(ctxs, bp, up, n, float(tol), st)
    if rc < 0:
        raise CoarseError(rc, L.coarse_last_error(None).decode() if noalloc else "batch solve failed")
    return outs, [{f: getattr(s, f) for f, _ in _Stats._fields_} for s in st]


class Batch:
    """Lock-step batch of independent solves (continuous batching): solves join with
    :meth:`submit` and leave when :meth:`step` reports them finished. All dense local
    and reduced solves of the live solves run in one GEMV launch per iteration.

    ``stream``: a ``torch.cuda.Stream`` ordering the batch against the caller (the
    right-hand sides must be ready on it); ``use_graph`` replays one captured lock
    step as a HIP graph (needs a non-default stream)."""

    def __init__(self, stream=None, use_graph=False):
        import torch
        L = load()
        self._L = L
        self.stream = stream
        handle = ctypes.c_void_p(stream.cuda_stream) if stream is not None else ctypes.c_void_p(
            torch.cuda.current_stream().cuda_stream)
        bt = ctypes.c_void_p()
        rc = L.coarse_batch_create(handle, int(bool(use_graph)), ctypes.byref(bt))
        if rc != 0:
            raise CoarseError(rc, L.coarse_last_error(None).decode())
        self._bt = bt
        self._keep = {}

    def submit(self, solver, b, u, tag, tol=1e-8):
        rc = self._L.coarse_batch_submit(self._bt, solver._ctx, solver._vec(b), solver._vec(u), float(tol), int(tag))
        if rc != 0:
            raise CoarseError(rc, "batch submit failed")
        self._keep[int(tag)] = (solver, b, u)

    def step(self, iters=1, cap=4096):
        """Advance every live solve by ``iters`` iterations; returns [(tag, stats)] of
        the solves that finished."""
        tags = (ctypes.c_int64 * cap)()
        st = (_Stats * cap)()
        nd = ctypes.c_int(0)
        rc = self._L.coarse_batch_step(self._bt, int(iters), tags, st, int(cap), ctypes.byref(nd))
        if rc != 0:
            raise CoarseError(rc, "batch step failed")
        return self._retired(tags, st, nd)

    def launch(self, iters=1):
        """First half of :meth:`step`: queue ``iters`` iterations of every live solve
        and return at once (no submit until :meth:`collect`)."""
        rc = self._L.coarse_batch_launch(self._bt, int(iters))
        if rc != 0:
            raise CoarseError(rc, "batch launch failed")

    def collect(self, cap=4096):
        """Second half of :meth:`step`: wait for the launched iterations; returns
        [(tag, stats)] of the solves that finished ([] when nothing was launched)."""
        tags = (ctypes.c_int64 * cap)()
        st = (_Stats * cap)()
        nd = ctypes.c_int(0)
        rc = self._L.coarse_batch_collect(self._bt, tags, st, int(cap), ctypes.byref(nd))
        if rc != 0:
            raise CoarseError(rc, "batch collect failed")
        return self._retired(tags, st, nd)

    def _retired(self, tags, st, nd):
        out = []
        for k in range(nd.value):
            d = {f: getattr(st[k], f) for f, _ in _Stats._fields_}
            d["code"] = d["status"]
            out.append((int(tags[k]), d))
            self._keep.pop(int(tags[k]), None)
        return out

    @property
    def live(self):
        return int(self._L.coarse_batch_live(self._bt))

    def close(self):
        if getattr(self, "_bt", None):
            self._L.coarse_batch_destroy(self._bt)
            self._bt = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
