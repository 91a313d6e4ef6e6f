"""Benchmark: coarse solves per second to a 1e-8 relative residual on one MI355X.

One step = one full PCG solve of the coarse Q1 Poisson system A u = b with the
two-level additive Schwarz preconditioner (every row of the hot path: A apply,
R_p gather, batched dense local and reduced solves, J^T / J, overlap sum, PCG
vector ops) on the mixed-versus-FP64 workload: the 128^3 quarter annulus (2.1M
elements, radial stretching 1.05, randomly renumbered), 4096 subdomains of 8^3
elements with one layer of overlap, 16 boxes per axis (17^3 reduced grid),
Dirichlet on r = 1, RHS i.i.d. N(0,1) (a different seeded RHS per step, up to 8
distinct ones). Inputs are resident on the GPU before timing; the per-mesh setup
(factorisations) is done once before the timed region and reported separately.

Prints one JSON line. The FP64 solve rate is `value`; the two mixed forms are
reported beside it (FP32 local/reduced inverses and interpolation, and the same
with the inverses stored in FP16; both keep the operator, residual, dot products
and outer iteration in FP64), each with p50/p99 latency. Also reported: the
64^3 cube (one GPU's share of a larger problem) with its own oracle baseline,
the 64-mesh batched workload, the preconditioner ablations, serving over
resident contexts, the warm start and the 16-right-hand-side block solve.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else float("nan")


GEMV_PHASE = 3

# HBM bytes per dense-solve launch (k_gemv_whole_f64) per workload from hardware counters
# (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, per dispatch, scaled by the same
# counters read on a 1 GiB device copy: FETCH x2.0, WRITE x1.0), and the
# fingerprint of the GEMV source they were taken on. A changed kernel reports
# traffic as unknown until the counters are taken again.
GEMV_TRAFFIC = {
    "cube64": {"bytes": 1142724477, "fetch_kib": 556498.375, "write_kib": 2987.3125, "fetch_scale": 2.0,
               "write_scale": 1.0, "src": "ac0df0b104ed37dc"},
    "annulus128": {"bytes": 9236706440, "fetch_kib": 4498570.688, "write_kib": 23424.031, "fetch_scale": 2.0,
                   "write_scale": 1.0, "src": "ac0df0b104ed37dc"},
}


def _gemv_source_fingerprint():
    import hashlib
    path = os.path.join(ROOT, "paper_2606_20496_amd", "csrc", "kernels.hip")
    src = open(path).read()
    i = src.index("void k_gemv_f64(")
    a = src.rindex("\n// ----", 0, src.rindex("// ----", 0, i))
    b = src.index("__global__", i)
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def _traffic(workload):
    t = GEMV_TRAFFIC.get(workload)
    return t["bytes"] if t and _gemv_source_fingerprint() == t["src"] else None


def run_form(torch, coarse, mesh, rhs, precision, steps, warmup, tol, local_iters=0, **solver_kw):
    """Set up once, then time `steps` solves, each on its own right-hand side (all
    resident on the GPU). Only the dominant kernel is bracketed by HIP events in
    the timed region; a separate pass afterwards times every phase. local_iters
    > 0: inexact local solves (that many Jacobi-PCG steps per subdomain), whose
    launch is then the one timed."""
    # setup in its two halves: the host plan, then the device half (timed twice
    # from the same plan: the first in a process also pays one-time costs)
    t0 = time.perf_counter()
    plan = coarse.Plan.from_mesh(mesh, precision=precision, local_iters=local_iters, **solver_kw)
    t_plan = time.perf_counter() - t0
    t_dev = []
    for rep in range(2):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        S = coarse.CoarseSolver.from_plan(plan)
        torch.cuda.synchronize()
        t_dev.append(time.perf_counter() - t1)
        if rep == 0:
            S.close()
    plan.close()
    t_setup = t_plan + t_dev[0]
    u = torch.empty_like(rhs[0])
    for i in range(warmup):
        S.solve(rhs[i % len(rhs)], tol, out=u)
    torch.cuda.synchronize()
    lat, iters, worst = [], [], 0.0
    S.profile_start(1 << GEMV_PHASE)
    t_start = time.perf_counter()
    for i in range(steps):
        t1 = time.perf_counter()
        _, st = S.solve(rhs[(warmup + i) % len(rhs)], tol, out=u)
        lat.append(time.perf_counter() - t1)
        iters.append(st["iters"])
        worst = max(worst, st["relres_true"])
    torch.cuda.synchronize()
    # a solve of k iterations applies the preconditioner k times; launches after
    # convergence (at most a check interval) exit at once and do no work
    work_launches = int(sum(iters))
    elapsed = time.perf_counter() - t_start
    gemv = S.profile_stop()
    S.profile_start(0xFF)
    for i in range(2):
        S.solve(rhs[i], tol, out=u)
    phases = S.profile_stop()
    info = dict(S.info)
    S.close()
    return {
        "solves_per_s": steps / elapsed, "ms_per_solve": 1e3 * elapsed / steps,
        "p50_ms": 1e3 * _pct(lat, 50), "p99_ms": 1e3 * _pct(lat, 99),
        "iters": int(np.median(iters)), "iters_min": int(min(iters)), "iters_max": int(max(iters)),
        "relres_true_max": worst, "setup_s": t_setup, "plan_s": t_plan, "device_setup_s": t_dev, "info": info,
        "gemv": gemv[coarse.PHASES[GEMV_PHASE]], "gemv_work_launches": work_launches, "phases": phases,
    }


def _form_summary(f, dtype, precision):
    if f is None:
        return None
    avg_ms = f["gemv"][0] / max(f["gemv_work_launches"], 1)
    lb = local_inv_bytes(f["info"], precision)
    return {"value": round(f["solves_per_s"], 3), "unit": "solves/s", "dtype": dtype,
            "ms_per_step": round(f["ms_per_solve"], 4), "p50_ms": round(f["p50_ms"], 4),
            "p99_ms": round(f["p99_ms"], 4), "iters": f["iters"], "iters_range": [f["iters_min"], f["iters_max"]],
            "relres_true_max": f["relres_true_max"], "setup_s": round(f["setup_s"], 3),
            "plan_s": round(f["plan_s"], 3), "device_setup_ms": [round(1e3 * t, 2) for t in f["device_setup_s"]],
            "gemv_avg_launch_us": round(avg_ms * 1e3, 2), "gemv_alg_bytes": lb,
            "gemv_achieved_GBs": round(lb / (avg_ms / 1e3) / 1e9, 1)}


def inexact_launch_bytes(info, precision):
    """Bytes one launch of the inexact local solves must move: the stored A_p
    (ELL values and column words, FP64 diagonals) read once, whatever the number
    of steps (each row stays in registers), r_p read and z_p written per packed
    entry."""
    return info["local_bytes"] + info["sum_np"] * ((8 if precision == "fp64" else 4) + 8)


def run_inexact(torch, coarse, mesh, rhs, exact, ks, steps, warmup, tol, precisions=("fp64", "mixed")):
    """Inexact local solves (k Jacobi-PCG steps per subdomain, flexible outer PCG)
    against the stored inverses of the same mesh: solves/s, iterations, the local
    launch's time, and iterations x bytes of the local solves (the bytes the local
    term reads per application times the iterations)."""
    out = {"note": "k steps of diagonally preconditioned CG per subdomain (A_p in ELL form, FP64 values; FP32 "
                   "values in the mixed form) in place of the stored inverses; flexible outer PCG",
           "exact": {}, "inexact": {}}
    for prec, f in exact.items():
        if f is None:
            continue
        lb = local_inv_bytes(f["info"], prec)
        out["exact"][prec] = {"value": round(f["solves_per_s"], 3), "iters": f["iters"],
                              "local_bytes_per_application": lb,
                              "iters_x_local_GB": round(f["iters"] * lb / 1e9, 2),
                              "local_launch_us": round(f["gemv"][0] / max(f["gemv_work_launches"], 1) * 1e3, 2),
                              "device_GB": round(f["info"]["device_bytes"] / 1e9, 3)}
    for prec in precisions:
        for k in ks:
            f = run_form(torch, coarse, mesh, rhs, prec, steps, warmup, tol, local_iters=k)
            lb = inexact_launch_bytes(f["info"], prec)
            us = f["gemv"][0] / max(f["gemv_work_launches"], 1) * 1e3
            out["inexact"][f"{prec}_k{k}"] = {
                "value": round(f["solves_per_s"], 3), "ms_per_step": round(f["ms_per_solve"], 4),
                "p50_ms": round(f["p50_ms"], 4), "p99_ms": round(f["p99_ms"], 4), "iters": f["iters"],
                "relres_true_max": f["relres_true_max"], "setup_s": round(f["setup_s"], 3),
                "device_setup_ms": [round(1e3 * t, 2) for t in f["device_setup_s"]],
                "ell_width": f["info"]["ell_width"], "local_bytes_per_application": lb,
                "iters_x_local_GB": round(f["iters"] * lb / 1e9, 2), "local_launch_us": round(us, 2),
                "local_launch_GBs": round(lb / us / 1e3, 1) if us > 0 else None,
                "device_GB": round(f["info"]["device_bytes"] / 1e9, 3)}
            _log(f"inexact {prec} k={k}: {f['solves_per_s']:.3f} solves/s, {f['iters']} iterations, "
                 f"local launch {us:.1f} us")
    return out


def run_batch_workload(torch, coarse, mg, tol, reps=3):
    """64 independent meshes (n log-uniform in [6, 48], blocks of 4/6/8 elements)
    solved together in lock step (one GEMV launch for all their local and reduced
    solves per iteration, HIP-graph replay), versus one at a time."""
    meshes = mg.batch_meshes(count=64)
    out = {"meshes": len(meshes), "elements": int(sum(m.n_elem for m in meshes))}
    for prec in ("mixed16", "mixed", "fp64"):
        t0 = time.perf_counter()
        solvers = [coarse.CoarseSolver.from_mesh(m, precision=prec) for m in meshes]
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            bs = [torch.tensor(m.b, device="cuda") for m in meshes]
            us = [torch.empty_like(b) for b in bs]
        stream.synchronize()
        bt = coarse.Batch(stream=stream, use_graph=True)
        best, failed = None, 0
        for rep in range(reps + 1):
            t1 = time.perf_counter()
            for k, S in enumerate(solvers):
                bt.submit(S, bs[k], us[k], tag=k, tol=tol)
            while bt.live:
                failed += sum(st["status"] != 0 for _, st in bt.step(2))
            stream.synchronize()
            dt = time.perf_counter() - t1
            if rep > 0:
                best = dt if best is None else min(best, dt)
        bt.close()
        t1 = time.perf_counter()
        for k, S in enumerate(solvers):
            failed += S.solve(bs[k], tol, out=us[k])[1]["status"] != 0
        torch.cuda.synchronize()
        seq = time.perf_counter() - t1
        for S in solvers:
            S.close()
        out[prec] = {"batched_solves_per_s": round(len(meshes) / best, 2),
                     "one_at_a_time_solves_per_s": round(len(meshes) / seq, 2),
                     "setup_s_total": round(t_setup, 3), "failed": int(failed)}
    return out


def run_serving_resident(torch, coarse, mg, tol, rates=(500.0, 2000.0, 8000.0, 32000.0), count=2048,
                         precision="mixed", block_min=8):
    """Open-loop serving over resident contexts: the 64 batch meshes are set up
    beforehand (both for the continuous-batching server, mixed precision, and for
    the plain FP64 one-at-a-time path); requests arrive as a Poisson stream at
    each rate, each for a uniformly drawn mesh with a fresh N(0,1) right-hand
    side (uploaded from the host inside the loop). Latency is arrival to result.
    Each rate runs three ways: the lock-step batch alone; the batch plus block
    solves of same-mesh requests that wait for their context; and FP64 one at a
    time."""
    from paper_2606_20496_amd import serve
    meshes = mg.batch_meshes(count=64)
    srv = serve.Server(budget_bytes=200e9, precision=precision, use_graph=True, step_iters=2)
    for k, m in enumerate(meshes):
        srv.preload(k, m)
    seq_cache = {k: coarse.CoarseSolver.from_mesh(m, precision="fp64") for k, m in enumerate(meshes)}
    torch.cuda.synchronize()
    out = {"meshes": len(meshes), "requests_per_rate": count, "precision": precision,
           "resident_bytes": srv.used, "block_min": block_min, "rates": {}}
    # warm-up pass (graph capture, allocator) outside the measured runs
    warm = serve.make_resident_requests(meshes, 4000.0, 128, seed=1)
    srv.run(warm)
    # the block solve's vectors of every context (allocated at its first use)
    for S in srv.cache.values():
        S.solve_multi(torch.zeros((1, S.n_vert), dtype=torch.float64, device="cuda"))
    srv.block_min = 2
    srv.run(warm)
    srv.block_min = 0
    serve.serve_sequential(warm[:32], tol=tol, cache=seq_cache)
    for rate in rates:
        reqs = serve.make_resident_requests(meshes, rate, count, seed=int(rate))
        rec, wall = srv.run(reqs)
        served = serve.summarize(rec, wall)
        # the same server with block solves for same-mesh requests that wait
        # (block_min or more), stepped beside the lock steps
        srv.block_min = block_min
        rec3, wall3 = srv.run(reqs)
        srv.block_min = 0
        blocked = serve.summarize(rec3, wall3)
        rec2, wall2 = serve.serve_sequential(reqs, tol=tol, cache=seq_cache)
        seq = serve.summarize(rec2, wall2)
        keep = ("solves_per_s", "p50_ms", "p99_ms", "mean_iters", "max_relres_true", "failed")
        out["rates"][str(int(rate))] = {"batched_" + precision: {k: served[k] for k in keep},
                                        "batched_block_" + precision: {k: blocked[k] for k in keep},
                                        "one_at_a_time_fp64": {k: seq[k] for k in keep}}
        _log(f"serving rate {rate}: batched {served['solves_per_s']:.0f}/s p99 {served['p99_ms']:.1f} ms; "
             f"with block solves {blocked['solves_per_s']:.0f}/s p99 {blocked['p99_ms']:.1f} ms; "
             f"one-at-a-time {seq['solves_per_s']:.0f}/s p99 {seq['p99_ms']:.1f} ms")
    srv.close()
    for S in seq_cache.values():
        S.close()
    return out


def _dist(v):
    v = np.asarray(v, dtype=float)
    if not len(v):
        return None
    return {"n": int(v.size), "mean": round(float(v.mean()), 4), "p50": round(_pct(v, 50), 4),
            "p99": round(_pct(v, 99), 4)}


def run_serving_workload(torch, coarse, mg, tol, rates=(50.0, 2000.0), count=4096, budget_gb=64.0,
                         precision="mixed", plan_workers=12, sequential=True, projection=0, local_iters=0,
                         graph_off=False):
    """The serving workload with setups in the loop: Poisson arrivals at each rate,
    `count` requests, each a coarse solve on a seeded mesh with n log-uniform in
    [8, 96] and a z stretch of up to 20, 30% of them reusing an earlier mesh with
    a new N(0,1) right-hand side. Meshes are generated when first needed (by the
    plan workers, counted in the latency). The continuous-batching server (mixed
    precision, FP64 outer iteration, admission by an HBM budget that binds,
    least-recently-used eviction) against the plain FP64 one-at-a-time path on
    the same stream with the same budget. Latency is arrival to result. With
    projection = l > 0 the batched server runs a second time with a basis of l
    prior solutions per cached mesh (Sec. 5), so that requests that reuse a mesh
    start from the projection onto its earlier solutions. With local_iters = k > 0
    it runs again with inexact local solves (k Jacobi-PCG steps per subdomain):
    no local inverses, so less device memory per mesh and a shorter setup."""
    from paper_2606_20496_amd import serve
    out = {"requests_per_rate": count, "n_range": [8, 96], "reuse": 0.3, "budget_GB": budget_gb,
           "precision": precision, "plan_workers": plan_workers, "rates": {}}
    keep_proj = ("solves_per_s", "p50_ms", "p99_ms", "mean_iters", "max_relres_true", "cache_misses", "failed",
                 "mean_iters_reused", "median_relres0_reused")
    keep = ("requests", "wall_s", "solves_per_s", "p50_ms", "p99_ms", "mean_iters", "max_relres_true",
            "cache_misses", "failed", "mean_iters_reused")
    for rate in rates:
        reqs = serve.make_requests(rate, count, lazy=True)
        srv = serve.Server(budget_gb * 1e9, precision=precision, use_graph=True, step_iters=2,
                           plan_workers=plan_workers)
        rec, wall = srv.run(reqs, progress=lambda m, r=rate: _log(f"serving {r:g} req/s: {m}"))
        summ = {k: v for k, v in serve.summarize(rec, wall).items() if k in keep}
        summ.update(evictions=srv.evictions, resolved=srv.resolved,
                    estimate_ratio_max=round(srv.estimate_ratio_max, 3),
                    setup_per_miss_s={k: _dist(v) for k, v in srv.setup_times.items()})
        srv.close()
        res = {"batched_" + precision: summ}
        _log(f"serving {rate:g} req/s: batched {summ['solves_per_s']:.1f}/s p50 {summ['p50_ms']:.0f} ms "
             f"p99 {summ['p99_ms']:.0f} ms, failed {summ['failed']}")
        variants = []
        if projection > 0:
            variants.append(("projected", {"projection": int(projection)}, True))
        if local_iters > 0:
            variants.append((f"inexact_k{int(local_iters)}", {"local_iters": int(local_iters)}, True))
        if graph_off:
            variants.append(("no_graph", {}, False))
            if local_iters > 0:
                variants.append((f"inexact_k{int(local_iters)}_no_graph", {"local_iters": int(local_iters)}, False))
        for name, kw, graph in variants:
            srv = serve.Server(budget_gb * 1e9, precision=precision, use_graph=graph, step_iters=2,
                               plan_workers=plan_workers, solver_kw=kw)
            rec3, wall3 = srv.run(reqs, progress=lambda m, r=rate, v=name: _log(f"serving {r:g} req/s, {v}: {m}"))
            pj = {k: v for k, v in serve.summarize(rec3, wall3).items() if k in keep_proj}
            pj.update(solver_kw=kw, use_graph=graph, evictions=srv.evictions,
                      setup_per_miss_s={k: _dist(v) for k, v in srv.setup_times.items()})
            srv.close()
            res[f"batched_{precision}_{name}"] = pj
            _log(f"serving {rate:g} req/s: {name} {pj['solves_per_s']:.1f}/s p50 {pj['p50_ms']:.0f} ms "
                 f"p99 {pj['p99_ms']:.0f} ms, mean iterations {pj['mean_iters']:.1f} against "
                 f"{summ['mean_iters']:.1f}, failed {pj['failed']}")
        if sequential is True or (sequential and rate in sequential):
            rec2, wall2 = serve.serve_sequential(reqs, tol=tol, budget_bytes=budget_gb * 1e9,
                                                 progress=lambda m, r=rate: _log(f"sequential {r:g}: {m}"))
            seq = {k: v for k, v in serve.summarize(rec2, wall2).items() if k in keep}
            res["one_at_a_time_fp64"] = seq
            _log(f"serving {rate:g} req/s: one at a time {seq['solves_per_s']:.1f}/s p99 {seq['p99_ms']:.0f} ms")
        out["rates"][str(int(rate))] = res
    return out


def c5_oracle_subset(torch, coarse, mg, tol, count=64, nmax=40, precision="mixed", rate=2000.0):
    """The serving workload's oracle check and CPU baseline on a seeded subset:
    the first `count` requests of the arrival stream whose mesh has n <= nmax
    (the oracle's setup of the largest meshes takes minutes), served together by
    the batched server, each checked against the FP64 oracle (iterations within
    the mixed forms' bar, solution within 1e-6), and the oracle's own rate on them
    (setup of each distinct mesh plus every solve, one at a time)."""
    import math as _m
    import os as _os
    from oracle import problem
    from paper_2606_20496_amd import serve
    t, mesh_id, rhs_seed = mg.serving_arrivals(rate, count=4096)
    picked, meshes = [], {}
    for q in range(len(t)):
        k = int(mesh_id[q])
        if mg.serving_request_n(k) > nmax:
            continue
        if k not in meshes:
            meshes[k] = mg.serving_request_mesh(k)
        picked.append(serve.Request(t_arrive=0.0, key=k, mesh=meshes[k], b=mg.rhs_normal(meshes[k], int(rhs_seed[q])),
                                    rid=q))
        if len(picked) == count:
            break
    srv = serve.Server(64e9, precision=precision, use_graph=True, step_iters=2, keep_outputs=True)
    rec, wall = srv.run(picked)
    srv.close()
    by = {r.rid: r for r in rec}
    probs, worst, t_setup, t_solve, iters_ok = {}, 0.0, 0.0, 0.0, True
    for rq in picked:
        t0 = time.perf_counter()
        if rq.key not in probs:
            probs[rq.key] = problem.from_mesh(rq.mesh)
        t1 = time.perf_counter()
        uo, io = probs[rq.key].solve(rq.b, tol=tol)
        t2 = time.perf_counter()
        t_setup += t1 - t0
        t_solve += t2 - t1
        r = by[rq.rid]
        u = r.u.detach().cpu().numpy()
        worst = max(worst, float(np.linalg.norm(u - uo) / np.linalg.norm(uo)))
        iters_ok &= r.status == 0 and r.iters <= max(_m.ceil(1.1 * io["iters"]), io["iters"] + 2)
    cores = len(_os.sched_getaffinity(0))
    return {"requests": len(picked), "distinct_meshes": len(probs), "n_max": nmax,
            "served_solves_per_s": round(len(picked) / wall, 2),
            "oracle": {"value": round(len(picked) / (t_setup + t_solve), 4), "unit": "solves/s", "cores": cores,
                       "kind": "oracle", "setup_s": round(t_setup, 2), "solve_s": round(t_solve, 2)},
            "max_rel_err_u": worst, "iters_within_bar": bool(iters_ok)}


INV_ELEM_BYTES = {"fp64": 8, "mixed": 4, "mixed16": 2}


def local_inv_bytes(info, precision):
    """Stored inverse bytes the dense-solve launch on the context's stream reads:
    all of them, or the local inverses alone when a reduced system of more than
    48 tile rows is solved beside it on a second stream (timed as its own phase)."""
    if not info["reduced_stream"]:
        return info["inv_alg_bytes"]
    n_r = info["n_r"]
    return info["inv_alg_bytes"] - n_r * (n_r + 1) // 2 * INV_ELEM_BYTES[precision]


def kernel_bytes(info, n_elem, precision):
    """Algorithmic bytes per launch of the per-iteration kernels (what the method
    must move with this storage; index tables of the blocking scheme excluded):
    A+p  : A^e (28 off-diagonal FP64 = 224 B; its rows sum to zero) + 8 u16 slots
           per element; z, p_old read,
           p and q written per free vertex
    R_p+J^T: the convergence test, plus the first stage of J^T (per J entry vertex
           id, weight, 3 local coordinates and the r value) when the reduced system
           shares the local systems' stream, or the R_p gather (per packed entry
           index + r value + r_p write) for the inexact local solves; with stored
           inverses the dense solves gather r_p themselves, and with the reduced
           branch on the second stream the J^T stage runs there (no entry then)
    sum+J: per packed entry position + z_p; per free vertex cover pointer, r read,
           z written, J pointer; per J entry base corner, weight, 3 coordinates
    x,r update: x, r read and written, p, q read per free vertex."""
    es = 8 if precision == "fp64" else 4
    nf, snp, nj = info["n_free"], info["sum_np"], info["n_jent"]
    out = {
        "A+p": n_elem * (224 + 16) + nf * 32,
        "sum+J": snp * (4 + 8) + nf * (4 + 8 + 8 + 4) + nj * (4 + es + 3 * es),
        "x,r update": nf * 48,
    }
    if info.get("local_iters", 0) > 0:
        out["R_p+J^T"] = snp * (4 + 8 + es)
    elif not info.get("reduced_stream", 0):
        out["R_p+J^T"] = nj * (4 + es + 3 * es + 8)
    return out


def run_ablations(torch, coarse, mesh, b, tol, max_it=400):
    """Iterations to the tolerance for the preconditioner's parts and variants on
    the 64^3 cube (FP64): the additive two-level method, its local part alone,
    its reduced part alone, the symmetrised coarse-local-coarse hybrid, the
    paper's hybrid of eqs. (asm1)-(asm2) under the flexible beta, and two layers
    of overlap (the paper's study of the parts, Sec. 5)."""
    out = {}
    for name, kw in (("additive", {}), ("local_only", {"mode": "local_only"}),
                     ("reduced_only", {"mode": "reduced_only"}), ("hybrid_sym", {"mode": "hybrid_sym"}),
                     ("hybrid", {"mode": "hybrid"}), ("additive_overlap2", {"overlap": 2})):
        S = coarse.CoarseSolver.from_mesh(mesh, max_it=max_it, **kw)
        u = torch.empty_like(b)
        t0 = time.perf_counter()
        try:
            _, st = S.solve(b, tol, out=u)
            res = {"iters": st["iters"], "converged": st["code"] == 0, "relres": st["relres"]}
        except coarse.CoarseError as err:
            # the reduced part alone is singular on the full space: PCG breaks down
            res = {"iters": None, "converged": False, "error": str(err)}
        torch.cuda.synchronize()
        out[name] = {**res, "ms": round(1e3 * (time.perf_counter() - t0), 3), "device_bytes": S.device_bytes}
        S.close()
    return out


FP64_MFMA_PEAK_TFS = 78.6    # MI355X dense FP64 matrix peak
FP32_MFMA_PEAK_TFS = 157.3   # MI355X dense FP32 matrix peak


def run_multi(torch, coarse, mg, mesh, tol, steps, warmup, k=16, precision="fp64"):
    """Block solve (coarse_solve_multi) of k right-hand sides on the bench mesh:
    the load of the bench plus k - 1 bump loads, solved together. Host clock over
    `steps` block solves; HIP events around each dense-solve launch (k_m_gemv on
    the matrix cores: FP64, or FP32 for the mixed forms), whose algorithmic work
    is 2 n^2 k flops per system and the packed inverse bytes read once."""
    rhs = [mesh.b] + [mg.rhs_bumps(mesh, 300 + j) for j in range(1, k)]
    B = torch.stack([torch.tensor(b, device="cuda") for b in rhs])
    U = torch.empty_like(B)
    S = coarse.CoarseSolver.from_mesh(mesh, precision=precision)
    for _ in range(warmup):
        S.solve_multi(B, tol, out=U)
    torch.cuda.synchronize()
    S.profile_start(1 << GEMV_PHASE)
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = S.solve_multi(B, tol, out=U)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms, cnt = S.profile_stop()[coarse.PHASES[GEMV_PHASE]]
    info = dict(S.info)
    S.close()
    iters = [s["iters"] for s in st]
    # dense-solve launches with work per block solve: the start plus one per
    # iteration until the last column converges
    work = steps * (max(iters) + 1)
    avg_s = ms / max(work, 1) / 1e3
    sum_n = info["sum_np"] + info["n_r"]
    sum_n2 = info["inv_alg_bytes"] // (INV_ELEM_BYTES[precision] // 2) - sum_n   # from sum n(n+1)/2 * es bytes
    flops = 2 * sum_n2 * k
    peak = FP64_MFMA_PEAK_TFS if precision == "fp64" else FP32_MFMA_PEAK_TFS
    return {"k": k, "precision": precision, "solves_per_s": round(k * steps / elapsed, 2), "ms_per_block": round(1e3 * elapsed / steps, 3),
            "iters": iters, "relres_true_max": max(s["relres_true"] for s in st),
            "status": sorted({s["status"] for s in st}),
            "gemv": {"kernel": "k_m_gemv", "avg_launch_us": round(avg_s * 1e6, 2), "launches": cnt,
                     "work_launches": work, "alg_flops": flops,
                     "TFLOPs": round(flops / avg_s / 1e12, 2), "peak_TFLOPs": peak,
                     "frac_mfma": round(flops / avg_s / 1e12 / peak, 4),
                     "alg_bytes": info["inv_alg_bytes"],
                     "GBs": round(info["inv_alg_bytes"] / avg_s / 1e9, 1)}}


def run_warm_start(torch, coarse, mg, mesh, tol, steps=32, basis=8, precisions=("fp64", "mixed16")):
    """A sequence of `steps` right-hand sides from a load that changes smoothly in
    time (time step 0.005: features move about a third of an element per step at
    64^3), solved cold (u_0 = 0) and from the projection onto the last `basis`
    solutions (Sec. 5). Host-clock ms per solve, iterations, and the initial
    residual the projection leaves."""
    bs = [torch.tensor(b, device="cuda") for b in mg.rhs_sequence(mesh, 777, steps)]
    out = {"steps": steps, "basis": basis, "dt": 0.005}
    for prec in precisions:
        S = coarse.CoarseSolver.from_mesh(mesh, precision=prec, projection=basis)
        u = torch.empty_like(bs[0])
        res = {}
        for form, fn in (("cold", S.solve), ("projected", S.solve_projected)):
            S.projection_reset()
            fn(bs[0], tol, out=u)      # warm the kernels (and, projected, the first basis vector)
            S.projection_reset()
            torch.cuda.synchronize()
            iters, r0, worst = [], [], 0.0
            t0 = time.perf_counter()
            for b in bs:
                _, st = fn(b, tol, out=u)
                iters.append(st["iters"])
                r0.append(st["relres0"])
                worst = max(worst, st["relres_true"])
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            res[form] = {"ms_per_solve": round(1e3 * t / steps, 3), "iters_mean": round(float(np.mean(iters)), 2),
                         "iters_first": iters[0], "iters_last": iters[-1],
                         "relres0_median": float(np.median(r0)), "worst_relres_true": worst}
        res["speedup"] = round(res["cold"]["ms_per_solve"] / res["projected"]["ms_per_solve"], 3)
        out[prec] = res
        S.close()
    return out


def _host():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = "unknown"
    try:
        b = np.show_config(mode="dicts")["Build Dependencies"]["blas"]
        blas = f"{b.get('name', '?')} {b.get('version', '')}".strip()
    except Exception:  # noqa: BLE001
        pass
    return {"cores": len(os.sched_getaffinity(0)), "cpu_model": model, "blas": blas}


def cpu_baseline_cube64(mesh, tol, runs=3):
    """The FP64 oracle, as it stands, on the host cores: full solves of the 64^3
    workload's first right-hand side (setup timed separately and excluded),
    median of `runs`."""
    from oracle import problem
    t0 = time.perf_counter()
    P = problem.from_mesh(mesh)
    t_setup = time.perf_counter() - t0
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        u, info = P.solve(mesh.b, tol=tol)
        ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    h = _host()
    return {"value": round(1.0 / t, 4), "unit": "solves/s", "cores": h["cores"], "kind": "oracle",
            "sample": f"full FP64 PCG solves of the 64^3 workload (first RHS), median of {runs} "
                      f"({info['iters']} iterations, {t:.2f} s; oracle setup {t_setup:.1f} s excluded)",
            "iters": info["iters"], "setup_s": round(t_setup, 2), "cpu_model": h["cpu_model"], "blas": h["blas"]}


C3_GOLDEN = os.path.join(ROOT, "tests", "golden", "c3_oracle.json")


def cpu_baseline_c3(mesh, n_local=256, iters=2):
    """The FP64 oracle, as it stands, on a bounded sample of the 128^3 annulus
    solve: its own routines time the work of one PCG iteration there (the
    operator product, the local solves of `n_local` of the 4096 subdomains,
    scaled to all of them, the reduced solve, the vector updates), and the rate
    is one solve of the oracle's iteration count at that cost. The oracle's setup
    of the sampled parts is excluded; its full setup of this workload is not run
    (minutes; the stored oracle solve records it)."""
    from oracle import fem, reduced, schwarz
    with open(C3_GOLDEN) as f:
        golden = json.load(f)
    d = mesh.dirichlet.astype(bool)
    t0 = time.perf_counter()
    A, Ae, _, free, fidx = fem.stiffness(mesh.xyz, mesh.e2v, d)
    mult = fem.multiplicity(mesh.e2v, mesh.n_vert)
    red = reduced.CentroidSpace(mesh.xyz, mesh.e2v, d, Ae, mesh.boxes, fidx, mult)
    sel = np.sort(np.random.default_rng(0).choice(mesh.n_part, n_local, replace=False))
    part = np.asarray(mesh.part)
    keep = np.isin(part, sel)
    # the sampled subdomains' overlapping sets and R_p (element layers are grown
    # over the whole mesh, so the sets equal those of the full construction)
    sets = schwarz.overlapping_subdomains(mesh.e2v, np.where(keep, np.searchsorted(sel, part), n_local),
                                          n_local + 1, 1)[:n_local]
    R = [fidx[r] for r in schwarz.restriction_sets(mesh.e2v, sets, d)]
    loc = schwarz.LocalSolves(A, R)
    t_setup = time.perf_counter() - t0
    rng = np.random.default_rng(1)
    r = rng.standard_normal(free.size)
    p = rng.standard_normal(free.size)
    x = np.zeros(free.size)
    ts = []
    for _ in range(iters):
        t0 = time.perf_counter()
        q = A @ p                          # operator
        alpha = float(r @ r) / float(p @ q)
        x += alpha * p                     # vector updates
        r -= alpha * q
        t_vec0 = time.perf_counter()
        z = loc.apply(r)                   # sampled local solves
        t_loc = time.perf_counter() - t_vec0
        t1 = time.perf_counter()
        z = z + red.apply(r)               # reduced solve
        beta = float(r @ z) / float(r @ r)
        p = z + beta * p
        t_other = time.perf_counter() - t1 + (t_vec0 - t0)
        ts.append(t_other + t_loc * mesh.n_part / n_local)
    t_iter = float(np.median(ts))
    n_it = int(golden["iters"])
    h = _host()
    return {"value": round(1.0 / (t_iter * n_it), 5), "unit": "solves/s", "cores": h["cores"], "kind": "oracle",
            "sample": f"oracle routines timing one PCG iteration of the 128^3 annulus workload (operator, local "
                      f"solves of {n_local} of {mesh.n_part} subdomains scaled to all, reduced solve, vector "
                      f"updates; median of {iters}), times the oracle's {n_it} iterations; sampled setup "
                      f"{t_setup:.1f} s excluded",
            "s_per_iter": round(t_iter, 4), "iters": n_it, "cpu_model": h["cpu_model"], "blas": h["blas"],
            "full_oracle_solve_s_stored": golden.get("oracle_solve_s"),
            "full_oracle_host_stored": golden.get("host")}


def run_ablations_c1(mesh, tol):
    """Iterations of the preconditioner's parts and variants on the 8^3 cube from
    the oracle (the GPU reaches the same counts; tested)."""
    from oracle import problem
    out = {}
    for name, kw, flex in (("additive", {}, False), ("local_only", {"mode": "local_only"}, False),
                           ("hybrid_sym", {"mode": "hybrid_sym"}, False), ("hybrid", {"mode": "hybrid"}, True),
                           ("additive_overlap2", {"overlap": 2}, False)):
        P = problem.from_mesh(mesh, **kw)
        u, info = P.solve(mesh.b, tol=tol, flexible=flex)
        out[name] = {"iters": info["iters"], "converged": bool(info["converged"])}
    return out


def _kernel_table(coarse, f, n_elem, precision):
    kb = kernel_bytes(f["info"], n_elem, precision)
    ks = {}
    for name, (ms, cnt) in f["phases"].items():
        avg = ms / max(cnt, 1) * 1e3
        e = {"avg_us": round(avg, 2), "launches": cnt}
        if name in kb and avg > 0:
            gbs = kb[name] / (avg * 1e-6) / 1e9
            e.update(alg_bytes=kb[name], GBs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))
        ks[name] = e
    return ks


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--n", type=int, default=128, help="annulus edge in elements (128 = the mixed-vs-FP64 mesh)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cube64", action="store_true", help="skip the 64^3 cube forms and their oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-mesh batched workload")
    ap.add_argument("--no-ablations", action="store_true", help="skip the preconditioner-part study")
    ap.add_argument("--no-warm-start", action="store_true", help="skip the successive right-hand-side study")
    ap.add_argument("--no-multi", action="store_true", help="skip the 16-right-hand-side block solve")
    ap.add_argument("--no-inexact", action="store_true", help="skip the inexact local solves study")
    ap.add_argument("--inexact-k", default="4,8,12", help="Jacobi-PCG steps per subdomain of the inexact study")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the open-loop serving study over resident contexts")
    ap.add_argument("--serving", action="store_true", help="also run the serving workload with setups in the loop")
    ap.add_argument("--serving-rates", default="50,2000", help="arrival rates (req/s) of --serving")
    ap.add_argument("--serving-count", type=int, default=4096, help="requests per rate of --serving")
    ap.add_argument("--serving-no-sequential", action="store_true",
                    help="skip the FP64 one-at-a-time comparison of --serving")
    ap.add_argument("--serving-sequential-rates", default="",
                    help="run the FP64 one-at-a-time comparison at these rates only (default: every rate)")
    ap.add_argument("--serving-projection", type=int, default=0,
                    help="also run --serving with a basis of this many prior solutions per cached mesh")
    ap.add_argument("--serving-local-iters", type=int, default=0,
                    help="also run --serving with inexact local solves of this many steps")
    ap.add_argument("--serving-graph-off", action="store_true",
                    help="also run --serving without graph replay of the lock step")
    ap.add_argument("--serving-oracle-subset", type=int, default=64,
                    help="requests of the seeded oracle subset of --serving (0: none)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run a plain 1 GiB device copy (known bytes) to scale HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design, not a measured configuration.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_20496_amd import coarse, meshgen as mg

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    coarse.load()
    if args.copy_calib:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- headline: the 128^3 quarter annulus, FP64 and the two mixed forms ----
    _log(f"annulus{args.n}: mesh")
    mesh = mg.large_annulus(n=args.n)
    workload = f"annulus{args.n}"
    nrhs = min(args.steps + args.warmup, 8)
    rhs = [torch.tensor(mesh.b if i == 0 else mg.rhs_normal(mesh, 100 + i), device="cuda") for i in range(nrhs)]
    _log("fp64 form")
    fp64 = run_form(torch, coarse, mesh, rhs, "fp64", args.steps, args.warmup, args.tol)
    _log(f"fp64: {fp64['solves_per_s']:.3f} solves/s, {fp64['iters']} iterations")
    mixed = mixed16 = mixed16r = None
    if not args.no_mixed:
        mixed = run_form(torch, coarse, mesh, rhs, "mixed", args.steps, args.warmup, args.tol)
        _log(f"mixed: {mixed['solves_per_s']:.3f} solves/s, {mixed['iters']} iterations")
        mixed16 = run_form(torch, coarse, mesh, rhs, "mixed16", args.steps, args.warmup, args.tol)
        _log(f"mixed16: {mixed16['solves_per_s']:.3f} solves/s, {mixed16['iters']} iterations")
        mixed16r = run_form(torch, coarse, mesh, rhs, "mixed16", args.steps, args.warmup, args.tol, reduced_refine=1)
        _log(f"mixed16, refined reduced solve: {mixed16r['solves_per_s']:.3f} solves/s, {mixed16r['iters']} iterations")
    inexact = None
    ks = tuple(int(x) for x in args.inexact_k.split(",") if x)
    if not args.no_inexact and ks:
        _log("inexact local solves")
        inexact = {workload: run_inexact(torch, coarse, mesh, rhs,
                                         {"fp64": fp64, "mixed": mixed, "mixed16": mixed16}, ks,
                                         args.steps, args.warmup, args.tol,
                                         precisions=("fp64",) if args.no_mixed else ("fp64", "mixed"))}
    del rhs

    # roofline of the dominant kernel: the batched dense solve of the local systems
    # (symmetric GEMV over their stored inverses, one workgroup per system), HBM-bound
    ms, cnt = fp64["gemv"]
    avg_s = ms / max(fp64["gemv_work_launches"], 1) / 1e3
    alg_bytes = local_inv_bytes(fp64["info"], "fp64")
    achieved = alg_bytes / avg_s / 1e9 if avg_s > 0 else 0.0
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": _traffic(workload),
            "kernel": "k_gemv_whole_f64", "avg_launch_us": round(avg_s * 1e6, 2),
            "launches": cnt, "work_launches": fp64["gemv_work_launches"],
            "alg_bytes_per_launch": alg_bytes}
    kernels = {"fp64": _kernel_table(coarse, fp64, mesh.n_elem, "fp64")}
    if mixed is not None:
        kernels["mixed"] = _kernel_table(coarse, mixed, mesh.n_elem, "mixed")
        kernels["mixed16"] = _kernel_table(coarse, mixed16, mesh.n_elem, "mixed16")

    cpu = None
    if not args.no_cpu_baseline and args.n == 128:
        _log("cpu baseline (oracle, sampled iteration of the 128^3 annulus)")
        cpu = cpu_baseline_c3(mesh)
        _log(f"cpu baseline: {cpu['value']} solves/s ({cpu['s_per_iter']} s per iteration)")
    mesh_info = {"n_elem": mesh.n_elem, "n_free": mesh.n_free, "n_sub": fp64["info"]["n_sub"],
                 "n_r": fp64["info"]["n_r"]}
    del mesh

    # ---- the 64^3 cube: one GPU's share of a larger problem ----
    cube = None
    c2 = mg.gpu_share_cube()
    if not args.no_cube64:
        _log("cube64 forms")
        nr2 = min(20 + 3, 32)
        rhs2 = [torch.tensor(c2.b if i == 0 else mg.rhs_bumps(c2, 100 + i), device="cuda") for i in range(nr2)]
        cube = {"workload": "cube64: 64^3 jittered Q1 hex cube, randomly renumbered, Dirichlet x=0; 512 "
                            "subdomains of 8^3 elements, overlap 1; 8^3 boxes; RHS 20 Gaussian bumps + noise"}
        c2_fp64 = run_form(torch, coarse, c2, rhs2, "fp64", 20, 3, args.tol)
        cube["fp64"] = _form_summary(c2_fp64, "f64", "fp64")
        cube["kernels_fp64"] = _kernel_table(coarse, c2_fp64, c2.n_elem, "fp64")
        ms2, _ = c2_fp64["gemv"]
        avg2 = ms2 / max(c2_fp64["gemv_work_launches"], 1) / 1e3
        lb2 = local_inv_bytes(c2_fp64["info"], "fp64")
        cube["fp64"]["roofline"] = {"kernel": "k_gemv_whole_f64", "avg_launch_us": round(avg2 * 1e6, 2),
                                    "alg_bytes_per_launch": lb2, "frac": round(lb2 / avg2 / 1e9 / HBM_PEAK_GBS, 4),
                                    "traffic": _traffic("cube64")}
        c2_mixed = c2_mixed16 = None
        if not args.no_mixed:
            c2_mixed = run_form(torch, coarse, c2, rhs2, "mixed", 20, 3, args.tol)
            c2_mixed16 = run_form(torch, coarse, c2, rhs2, "mixed16", 20, 3, args.tol)
            cube["mixed"] = _form_summary(c2_mixed, "f32", "mixed")
            cube["mixed16"] = _form_summary(c2_mixed16, "f16-stored", "mixed16")
        if inexact is not None:
            inexact["cube64"] = run_inexact(torch, coarse, c2, rhs2,
                                            {"fp64": c2_fp64, "mixed": c2_mixed, "mixed16": c2_mixed16}, ks,
                                            20, 3, args.tol,
                                            precisions=("fp64",) if args.no_mixed else ("fp64", "mixed"))
        if not args.no_cpu_baseline:
            _log("cube64 cpu baseline (oracle, median of 3)")
            cube["cpu_baseline"] = cpu_baseline_cube64(c2, args.tol)
        _log(f"cube64: fp64 {cube['fp64']['value']} solves/s")
        del rhs2

    batch = None
    if not args.no_batch:
        _log("batch workload")
        batch = run_batch_workload(torch, coarse, mg, args.tol)
        _log(f"batch: {batch}")
    ablations = None
    if not args.no_ablations:
        _log("ablations")
        b2 = torch.tensor(c2.b, device="cuda")
        ablations = {"cube64": run_ablations(torch, coarse, c2, b2, args.tol),
                     "cube8_oracle": run_ablations_c1(mg.small_cube(), args.tol)}
        _log(f"ablations: { {k: v['iters'] for k, v in ablations['cube64'].items()} }")

    resident = None
    if not args.no_serving:
        _log("serving over resident contexts")
        resident = run_serving_resident(torch, coarse, mg, args.tol)

    warm = None
    if not args.no_warm_start:
        _log("warm start")
        warm = run_warm_start(torch, coarse, mg, c2, args.tol)
        _log(f"warm start: {warm}")

    multi = None
    if not args.no_multi:
        _log("block solve, 16 right-hand sides")
        multi = run_multi(torch, coarse, mg, c2, args.tol, 5, 1)
        if cube is not None:
            multi["vs_single_fp64"] = round(multi["solves_per_s"] / cube["fp64"]["value"], 2)
        if not args.no_mixed:
            m16 = run_multi(torch, coarse, mg, c2, args.tol, 5, 1, precision="mixed16")
            if cube is not None:
                m16["vs_single_mixed16"] = round(m16["solves_per_s"] / cube["mixed16"]["value"], 2)
            multi["mixed16"] = m16
        _log(f"block solve: {multi}")

    serving = None
    if args.serving:
        _log("serving workload with setups in the loop")
        serving = run_serving_workload(torch, coarse, mg, args.tol,
                                       rates=tuple(float(x) for x in args.serving_rates.split(",")),
                                       count=args.serving_count,
                                       sequential=(False if args.serving_no_sequential else
                                                   {float(x) for x in args.serving_sequential_rates.split(",")}
                                                   if args.serving_sequential_rates else True),
                                       projection=args.serving_projection,
                                       local_iters=args.serving_local_iters, graph_off=args.serving_graph_off)
        if args.serving_oracle_subset > 0 and not args.no_cpu_baseline:
            _log("serving: oracle subset")
            serving["oracle_subset"] = c5_oracle_subset(torch, coarse, mg, args.tol, count=args.serving_oracle_subset)
            _log(f"serving oracle subset: {serving['oracle_subset']}")

    line = {
        "metric": "coarse solves/sec to 1e-8 rel. residual (mixed vs FP64); p50/p99 latency",
        "value": round(fp64["solves_per_s"], 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fp64["ms_per_solve"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{workload}: {args.n}^3 quarter annulus r in [1,2], theta in [0,pi/2], "
                               f"z in [0,1], radial ratio 1.05, jitter 0.05, randomly renumbered, Dirichlet r=1; "
                               f"{mesh_info['n_sub']} subdomains of 8^3 elements, overlap 1; {args.n // 8}^3 "
                               f"boxes; RHS N(0,1); PCG to {args.tol:g}", **mesh_info},
        "p50_ms": round(fp64["p50_ms"], 4),
        "p99_ms": round(fp64["p99_ms"], 4),
        "iters": fp64["iters"],
        "iters_range": [fp64["iters_min"], fp64["iters_max"]],
        "relres_true_max": fp64["relres_true_max"],
        "setup_s": round(fp64["setup_s"], 3), "plan_s": round(fp64["plan_s"], 3),
        "device_setup_ms": [round(1e3 * t, 2) for t in fp64["device_setup_s"]],
        "mixed": _form_summary(mixed, "f32 local/reduced inverses, f32 J, f64 operator/vectors/dots", "mixed"),
        "mixed16": _form_summary(mixed16, "f16 storage of the local/reduced inverses (power-of-two scale per "
                                          "system), f32 arithmetic, f32 J, f64 operator/vectors/dots", "mixed16"),
        "mixed16_refined": _form_summary(mixed16r, "mixed16 with one step of refinement of every reduced solve "
                                                   "(FP64 residual by the 27-point stencil of A_r)", "mixed16"),
        "kernels": kernels,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    for key, val in (("cube64", cube), ("inexact_local_solves", inexact), ("batch_workload", batch),
                     ("ablations", ablations),
                     ("warm_start", warm), ("multi_rhs", multi), ("serving_resident", resident),
                     ("serving_workload", serving)):
        if val is not None:
            line[key] = val
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
