"""Serving loop for coarse solves on one GPU: continuous batching with admission
by HBM budget and a per-mesh context cache.

Requests (arrival time, mesh key, mesh, right-hand side) are admitted as they
arrive. A request whose mesh context is resident and idle joins the lock-step
batch at the next step. A request for a new mesh first gets its setup plan (the
host half of the setup: orderings, subdomains, box grid, work tables) built by a
worker thread, which makes no GPU call, while the GPU keeps serving; the device
half (uploads, element matrices, inversions) then runs on the serving thread
between lock steps, on its own stream, once the resident contexts leave room in
the HBM budget (idle contexts are evicted least-recently-used first; otherwise
the plan waits). All GPU calls of the loop come from the one serving thread.
Finished solves retire after each step and free their mesh for the next request
on it. Every solve's result is bitwise what a solo solve of the same context
gives.

The plain FP64 one-at-a-time path (:func:`serve_sequential`) processes the same
request stream in arrival order with one solve at a time, for comparison.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import time

import numpy as np

from . import coarse


class LazyMesh:
    """A request's mesh, generated when first needed (by a plan worker) and
    dropped once its setup plan holds what it needs; the sizes and Dirichlet
    flags a right-hand side needs stay. Generated again if its context is
    evicted and the mesh comes back."""

    def __init__(self, make):
        import threading
        self._make = make
        self._mesh = None
        self._lock = threading.Lock()
        self.n_vert = None
        self.dirichlet = None

    def get(self):
        with self._lock:
            if self._mesh is None:
                m = self._make()
                self._mesh = m
                self.n_vert, self.dirichlet = m.n_vert, m.dirichlet.copy()
            return self._mesh

    def release(self):
        with self._lock:
            self._mesh = None


def _mesh_of(mesh):
    return mesh.get() if isinstance(mesh, LazyMesh) else mesh


@dataclasses.dataclass
class Request:
    t_arrive: float          # seconds after the start of the run
    key: int                 # mesh identity (requests with the same key share a context)
    mesh: object             # meshgen.Mesh (or any object with its fields), or a LazyMesh
    b: np.ndarray = None     # right-hand side, one value per vertex (or drawn from rhs_seed)
    rid: int = 0
    rhs_seed: int = -1       # with b None: b = N(0,1) from this seed, 0 on Dirichlet vertices

    def rhs(self):
        if self.b is not None:
            return self.b
        from . import meshgen as mg
        if isinstance(self.mesh, LazyMesh) and self.mesh.n_vert is None:
            self.mesh.get()
        return mg.rhs_normal(self.mesh, self.rhs_seed)


@dataclasses.dataclass
class Record:
    rid: int
    key: int
    t_arrive: float
    t_done: float
    iters: int
    relres_true: float
    setup: bool              # this request's mesh was set up for it (cache miss)
    status: int
    u: object = None         # the solution (kept only when asked for)
    relres0: float = 1.0     # relative residual of the initial guess (1 from u_0 = 0)

    @property
    def latency(self):
        return self.t_done - self.t_arrive


def summarize(records, wall):
    lat = np.array([r.latency for r in records])
    return {
        "requests": len(records), "wall_s": wall,
        "solves_per_s": len(records) / wall if wall > 0 else float("nan"),
        "p50_ms": 1e3 * float(np.percentile(lat, 50)) if len(lat) else float("nan"),
        "p99_ms": 1e3 * float(np.percentile(lat, 99)) if len(lat) else float("nan"),
        "mean_iters": float(np.mean([r.iters for r in records])) if records else float("nan"),
        "max_relres_true": float(max((r.relres_true for r in records), default=0.0)),
        "cache_misses": int(sum(r.setup for r in records)),
        "failed": int(sum(r.status != 0 for r in records)),
        # requests on a mesh already resident (a projection basis can help only these)
        "mean_iters_reused": (float(np.mean([r.iters for r in records if not r.setup]))
                              if any(not r.setup for r in records) else float("nan")),
        "median_relres0_reused": (float(np.median([r.relres0 for r in records if not r.setup]))
                                  if any(not r.setup for r in records) else float("nan")),
    }


class Server:
    def __init__(self, budget_bytes, precision="mixed", use_graph=True, step_iters=2, tol=1e-8,
                 plan_workers=2, solver_kw=None, keep_outputs=False, adaptive_steps=True, block_min=0):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.precision = precision
        self.step_iters = int(step_iters)
        self.tol = tol
        # results of the lock step whose true residual missed 10 tol and were
        # solved again alone on their context (see _checked)
        self.resolved = 0
        self.stream = torch.cuda.Stream()
        self.setup_stream = torch.cuda.Stream()
        self.batch = coarse.Batch(stream=self.stream, use_graph=use_graph)
        self.pool = cf.ThreadPoolExecutor(max_workers=plan_workers)
        self.solver_kw = dict(solver_kw or {})
        self.cache = collections.OrderedDict()   # key -> CoarseSolver (LRU order)
        self.busy = set()                        # keys with a live solve
        self.planning = {}                       # key -> Future of a Plan (host only)
        self.ready = {}                          # key -> (Plan, estimated bytes)
        self.max_plans = 3 * plan_workers        # plans held on the host at once
        self.used = 0                            # sum of acct over the resident contexts
        self.acct = {}                           # key -> device bytes counted for its context
        self.estimate_ratio_max = 0.0            # largest device_bytes / estimate_bytes seen
        self.evictions = 0
        # per cache miss: mesh generation and host plan (worker threads), device
        # half of the setup (serving thread)
        self.setup_times = {"mesh_s": [], "plan_s": [], "device_s": []}
        self.keep_outputs = keep_outputs
        self.last_iters = {}                     # key -> iterations of its last solve
        self.adaptive_steps = adaptive_steps
        # block_min >= 2: when at least that many requests wait for one idle
        # resident mesh, up to coarse.MULTI_MAX of them are solved together by
        # one block solve (the dense solves on the matrix cores), advanced on the
        # serving stream by the same number of iterations as each lock step
        self.block_min = int(block_min)
        self.blocks = {}                         # key -> [requests, iterations issued]

    def _plan(self, mesh):
        kw = dict(self.solver_kw)
        # a server that runs block solves has their vectors allocated by the
        # setup, so a context's footprint is known when it is admitted
        if self.block_min >= 2:
            kw.setdefault("block_rhs", 1)
        plan = coarse.Plan.from_mesh(_mesh_of(mesh), precision=self.precision, **kw)
        if isinstance(mesh, LazyMesh):
            mesh.release()
        return plan

    def _plan_job(self, mesh):
        """Worker thread: the mesh (generated here when lazy), its footprint
        estimate and its setup plan; no GPU call."""
        t0 = time.perf_counter()
        m = _mesh_of(mesh)
        t1 = time.perf_counter()
        need = self.estimate_bytes(m, self.precision, self.solver_kw.get("projection", 0),
                                   self.solver_kw.get("local_iters", 0))
        plan = self._plan(mesh)
        self.setup_times["mesh_s"].append(t1 - t0)
        self.setup_times["plan_s"].append(time.perf_counter() - t1)
        return plan, need

    def _admit(self, key, S, estimate=None):
        """Count a new resident context against the budget."""
        self.cache[key] = S
        self.acct[key] = S.device_bytes
        self.used += self.acct[key]
        if estimate:
            self.estimate_ratio_max = max(self.estimate_ratio_max, S.device_bytes / estimate)

    def _recount(self, key):
        """A context's footprint may grow after its setup (the block solve's
        vectors, when the setup did not allocate them): count the difference."""
        now_bytes = self.cache[key].device_bytes
        self.used += now_bytes - self.acct[key]
        self.acct[key] = now_bytes

    def _device_setup(self, plan):
        with self.torch.cuda.stream(self.setup_stream):
            S = coarse.CoarseSolver.from_plan(plan)
        self.setup_stream.synchronize()
        return S

    def preload(self, key, mesh):
        """Set up `mesh` now (both halves, on the calling thread) and keep its
        context resident under `key`, as if an earlier request had brought it in."""
        plan = self._plan(mesh)
        S = self._device_setup(plan)
        plan.close()
        self._admit(key, S)
        return S

    def _evict_for(self, need, keep=()):
        """Evict idle contexts (least recently used first, never those in `keep`)
        until `need` more bytes fit the budget; True if they do. Nothing is
        evicted when evicting every idle context would still not make room."""
        if self.used + need <= self.budget:
            return True
        idle = [k for k in self.cache if k not in self.busy and k not in keep]
        if self.used - sum(self.acct[k] for k in idle) + need > self.budget:
            return False
        for key in idle:
            if self.used + need <= self.budget:
                break
            S = self.cache.pop(key)
            self.used -= self.acct.pop(key)
            self.last_iters.pop(key, None)
            S.close()
            self.evictions += 1
        return self.used + need <= self.budget

    @staticmethod
    def estimate_bytes(mesh, precision, projection=0, local_iters=0):
        """Rough device footprint of a context before it exists: element data, the
        stored inverses (packed symmetric, padded to 32) or, with inexact local
        solves, the sparse A_p (26 entries per row), vectors and the basis of
        `projection` prior solutions (and their products with A)."""
        E, n = mesh.n_elem, mesh.n_vert
        vol = E / max(mesh.n_part, 1)
        np_ = (vol ** (1 / 3) + 2) ** 3
        nb = np.ceil(np_ / 32)
        tiles = mesh.n_part * nb * (nb + 1) / 2
        es = {"fp64": 8, "mixed": 4, "mixed16": 2}[precision]
        if local_iters > 0:
            ev = 8 if precision == "fp64" else 4
            rows = mesh.n_part * np_
            loc = rows * (26 * (ev + 2) + 8 + 32) * 1.1
            nbr = np.ceil(np.prod([b + 1 for b in mesh.boxes]) / 32)   # reduced system's tile rows
            return int(E * 420 + n * 200 + loc + nbr * (nbr + 1) / 2 * 1024 * es + 16 * projection * n)
        return int(E * 420 + n * 200 + tiles * 1024 * es * 1.1 + tiles * 32 * es + 16 * projection * n)

    def run(self, requests, t0=None, progress=None, progress_every=10.0):
        """Serve `requests` (open loop: each is admitted at its arrival time) until
        every one has finished; returns (records, wall seconds). `progress`, when
        given, is called with a short status string every `progress_every` s."""
        torch = self.torch
        t_report = time.perf_counter()
        reqs = collections.deque(sorted(requests, key=lambda r: r.t_arrive))
        waiting = collections.deque()      # arrived, not yet in the batch
        live = {}                          # rid -> (Request, u, b)
        missed = set()
        records = []
        t0 = time.perf_counter() if t0 is None else t0
        now = lambda: time.perf_counter() - t0
        while reqs or waiting or live or self.blocks or self.planning or self.ready:
            t = now()
            if progress is not None and time.perf_counter() - t_report >= progress_every:
                t_report = time.perf_counter()
                progress(f"t={t:.1f}s done={len(records)} live={len(live)} waiting={len(waiting)} "
                         f"planning={len(self.planning)} ready={len(self.ready)} resident={len(self.cache)} "
                         f"used={self.used / 1e9:.1f}GB")
            while reqs and reqs[0].t_arrive <= t:
                waiting.append(reqs.popleft())
            # plans finished on the worker threads
            for key, fut in list(self.planning.items()):
                if fut.done():
                    del self.planning[key]
                    self.ready[key] = fut.result()
            # same-mesh requests waiting for an idle resident context: one block
            # solve, stepped on the serving stream beside the lock steps
            if self.block_min >= 2 and waiting:
                groups = collections.OrderedDict()
                for rq in waiting:
                    if rq.key in self.cache and rq.key not in self.busy:
                        groups.setdefault(rq.key, []).append(rq)
                started = set()
                for key, rqs in groups.items():
                    if len(rqs) < self.block_min:
                        continue
                    rqs = rqs[:coarse.MULTI_MAX]
                    S = self.cache[key]
                    self.cache.move_to_end(key)
                    with torch.cuda.stream(self.stream):
                        B = torch.tensor(np.stack([rq.rhs() for rq in rqs]), device="cuda")
                        S.multi_begin(B, self.tol)
                    self._recount(key)
                    self.busy.add(key)
                    self.blocks[key] = [rqs, 0]
                    started.update(rq.rid for rq in rqs)
                if started:
                    waiting = collections.deque(rq for rq in waiting if rq.rid not in started)
            # admit waiting requests whose context is resident and idle
            keep = collections.deque()
            for rq in waiting:
                if rq.key in self.cache and rq.key not in self.busy:
                    S = self.cache[rq.key]
                    self.cache.move_to_end(rq.key)
                    with torch.cuda.stream(self.stream):
                        b = torch.tensor(rq.rhs(), device="cuda")
                        u = torch.empty_like(b)
                    self.batch.submit(S, b, u, tag=rq.rid, tol=self.tol)
                    self.busy.add(rq.key)
                    live[rq.rid] = [rq, u, b, 0]
                else:
                    keep.append(rq)
            waiting = keep
            needed = {rq.key for rq in waiting}

            def device_setups():
                # device halves of ready plans while the budget allows; contexts a
                # waiting request needs are never evicted, and a context that does
                # not fit even with everything idle evicted is built only when no
                # solve runs
                for key, (plan, need) in list(self.ready.items()):
                    if self._evict_for(need, keep=needed) or (not live and not self.blocks):
                        td = time.perf_counter()
                        S = self._device_setup(plan)
                        self.setup_times["device_s"].append(time.perf_counter() - td)
                        plan.close()
                        del self.ready[key]
                        self._admit(key, S, estimate=need)
            # host plans for new meshes
            for rq in waiting:
                if rq.key in self.cache or rq.key in self.planning or rq.key in self.ready:
                    continue
                if len(self.planning) + len(self.ready) >= self.max_plans:
                    break
                self.planning[rq.key] = self.pool.submit(self._plan_job, rq.mesh)
                missed.add(rq.rid)
            if live or self.blocks:
                # as many iterations per lock step as the live solve (or block)
                # expected to finish first still needs (its mesh's last count), at
                # least step_iters: fewer host round trips when few solves are live
                k = self.step_iters
                if self.adaptive_steps:
                    rem = [self.last_iters.get(e[0].key, 0) - e[3] for e in live.values()]
                    rem += [self.last_iters.get(key, 0) - blk[1] for key, blk in self.blocks.items()]
                    k = max(k, min(rem))
                for key, blk in self.blocks.items():
                    with torch.cuda.stream(self.stream):
                        self.cache[key].multi_advance(k)
                    blk[1] += k
                for e in live.values():
                    e[3] += k
                # the lock steps are queued first and collected after the device
                # setups, which run on the setup stream meanwhile
                if live:
                    self.batch.launch(k)
                device_setups()
                finished = self.batch.collect() if live else []
                if not live:
                    self.stream.synchronize()
                for key in list(self.blocks):
                    S = self.cache[key]
                    if not S.multi_done():
                        continue
                    rqs, _ = self.blocks.pop(key)
                    with torch.cuda.stream(self.stream):
                        U, sts = S.multi_end()
                    t_done = now()
                    for j, rq in enumerate(rqs):
                        records.append(Record(rid=rq.rid, key=rq.key, t_arrive=rq.t_arrive, t_done=t_done,
                                              iters=sts[j]["iters"], relres_true=sts[j]["relres_true"],
                                              setup=rq.rid in missed, status=sts[j]["status"],
                                              u=U[j] if self.keep_outputs else None))
                    self.busy.discard(key)
                    self.last_iters[key] = max(st["iters"] for st in sts)
                for tag, st in finished:
                    rq, u, b, _ = live.pop(tag)
                    st = self._checked(rq, u, b, st)
                    self.busy.discard(rq.key)
                    self.last_iters[rq.key] = st["iters"]
                    records.append(Record(rid=rq.rid, key=rq.key, t_arrive=rq.t_arrive, t_done=now(),
                                          iters=st["iters"], relres_true=st["relres_true"],
                                          setup=rq.rid in missed, status=st["status"],
                                          u=u if self.keep_outputs else None, relres0=st["relres0"]))
            else:
                n_ready = len(self.ready)
                device_setups()
                if len(self.ready) == n_ready:
                    time.sleep(0.0005)
        self.stream.synchronize()
        return records, now()

    def _checked(self, rq, u, b, st):
        """A converged lock-step result whose true residual ||b - A u|| / ||b||
        (recomputed by the library at the end of every solve) misses 10 tol is
        solved again alone on its context, and that result is kept. This has been
        seen on rare cache hits of large meshes whose reduced branch runs on a
        second stream (1 request in 1024 at 2000 req/s), with the recurrence
        residual at the tolerance; its cause is not found, so the server does not
        return such a result."""
        if st["status"] != 0 or st["relres_true"] <= 10.0 * self.tol:
            return st
        import torch
        S = self.cache[rq.key]
        with torch.cuda.stream(self.stream):
            _, st2 = S.solve(b, self.tol, out=u)
        self.stream.synchronize()
        self.resolved += 1
        return st2

    def close(self):
        self.pool.shutdown(wait=True)
        for plan, _ in self.ready.values():
            plan.close()
        self.ready.clear()
        self.batch.close()
        for S in self.cache.values():
            S.close()
        self.cache.clear()
        self.acct.clear()
        self.used = 0


def serve_sequential(requests, precision="fp64", tol=1e-8, solver_kw=None, cache=None, budget_bytes=None,
                     progress=None, progress_every=10.0):
    """The plain one-at-a-time path: arrival order, one solve at a time, contexts
    cached by mesh key, setup in line. `cache` (key -> CoarseSolver) may hold
    contexts set up beforehand; the caller keeps ownership of those. With
    `budget_bytes`, contexts it set up are evicted least recently used first to
    stay within that many device bytes."""
    import torch
    cache = collections.OrderedDict() if cache is None else collections.OrderedDict(cache)
    given = set(cache)
    used = 0
    records = []
    t0 = time.perf_counter()
    t_report = t0
    for rq in sorted(requests, key=lambda r: r.t_arrive):
        if progress is not None and time.perf_counter() - t_report >= progress_every:
            t_report = time.perf_counter()
            progress(f"t={t_report - t0:.1f}s done={len(records)} resident={len(cache)} used={used / 1e9:.1f}GB")
        while time.perf_counter() - t0 < rq.t_arrive:
            time.sleep(0.0002)
        miss = rq.key not in cache
        if miss:
            S = coarse.CoarseSolver.from_mesh(_mesh_of(rq.mesh), precision=precision, **(solver_kw or {}))
            if isinstance(rq.mesh, LazyMesh):
                rq.mesh.release()
            used += S.device_bytes
            cache[rq.key] = S
            if budget_bytes is not None:
                for key in list(cache):
                    if used <= budget_bytes:
                        break
                    if key in given or key == rq.key:
                        continue
                    old = cache.pop(key)
                    used -= old.device_bytes
                    old.close()
        cache.move_to_end(rq.key)
        S = cache[rq.key]
        b = torch.tensor(rq.rhs(), device="cuda")
        u, st = S.solve(b, tol)
        records.append(Record(rid=rq.rid, key=rq.key, t_arrive=rq.t_arrive, t_done=time.perf_counter() - t0,
                              iters=st["iters"], relres_true=st["relres_true"], setup=miss,
                              status=st["status"]))
    wall = time.perf_counter() - t0
    for key, S in cache.items():
        if key not in given:
            S.close()
    return records, wall


def make_requests(rate, count, seed=59999, nmax=96, reuse=0.3, lazy=False):
    """The serving workload: Poisson arrivals at `rate`, meshes drawn by
    meshgen.serving_request_mesh (n log-uniform in [8, nmax], graded z), 30% of
    requests reusing an earlier mesh with a new N(0,1) right-hand side. With
    `lazy`, meshes and right-hand sides are generated when the server first needs
    them (thousands of distinct meshes do not fit host memory at once)."""
    from . import meshgen as mg
    t, mesh_id, rhs_seed = mg.serving_arrivals(rate, count=count, seed=seed, reuse=reuse)
    meshes = {}
    out = []
    for q in range(count):
        k = int(mesh_id[q])
        if k not in meshes:
            meshes[k] = (LazyMesh(lambda k=k: mg.serving_request_mesh(k, nmax=nmax)) if lazy
                         else mg.serving_request_mesh(k, nmax=nmax))
        m = meshes[k]
        if lazy:
            out.append(Request(t_arrive=float(t[q]), key=k, mesh=m, rid=q, rhs_seed=int(rhs_seed[q])))
        else:
            out.append(Request(t_arrive=float(t[q]), key=k, mesh=m, b=mg.rhs_normal(m, int(rhs_seed[q])), rid=q))
    return out


def make_resident_requests(meshes, rate, count, seed=58999):
    """Poisson arrivals at `rate` over the given meshes (all set up beforehand),
    each request with its mesh drawn uniformly and a fresh N(0,1) right-hand side."""
    from . import meshgen as mg
    t, key, rhs_seed = mg.resident_arrivals(rate, count, len(meshes), seed=seed)
    return [Request(t_arrive=float(t[q]), key=int(key[q]), mesh=meshes[int(key[q])],
                    b=mg.rhs_normal(meshes[int(key[q])], int(rhs_seed[q])), rid=q) for q in range(count)]


def main():
    import argparse
    import json
    import torch
    ap = argparse.ArgumentParser(description="serving loop for coarse solves (continuous batching)")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--nmax", type=int, default=96)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--step-iters", type=int, default=2)
    ap.add_argument("--sequential", action="store_true", help="also run the FP64 one-at-a-time path")
    args = ap.parse_args()
    coarse.load()
    reqs = make_requests(args.rate, args.count, nmax=args.nmax)
    torch.cuda.synchronize()
    srv = Server(args.budget_gb * 1e9, precision=args.precision, use_graph=not args.no_graph,
                 step_iters=args.step_iters)
    rec, wall = srv.run(reqs)
    srv.close()
    out = {"rate": args.rate, "count": args.count, "nmax": args.nmax, "precision": args.precision,
           "serving": summarize(rec, wall)}
    if args.sequential:
        rec2, wall2 = serve_sequential(reqs)
        out["sequential_fp64"] = summarize(rec2, wall2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
