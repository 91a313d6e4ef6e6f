"""Benchmark: coarse solves per second to a 1e-8 relative residual on one MI355X.

One step = one full PCG solve of the coarse Q1 Poisson system A u = b, two-level
additive Schwarz preconditioned (every row of the hot path: A apply, R_p gather,
batched dense local and reduced solves, J^T / J, overlap sum, PCG vector ops), on
the one-GPU-share workload: the 64^3 jittered, randomly renumbered unit cube
(262,144 elements), 512 subdomains of 8^3 elements with one layer of overlap,
8 boxes per axis (9^3 reduced grid), RHS = 20 Gaussian bumps + noise (a
different seeded RHS per step, up to 32 distinct ones). Inputs are resident on
the GPU before timing; the per-mesh setup (factorisations) is done
once before the timed region and reported separately.

Prints one JSON line (rank 0). The FP64 solve rate is `value`. Two mixed forms
are reported beside it: FP32 local/reduced inverses and interpolation, and the
same with the inverses stored in FP16; both keep the operator, residual, dot
products and outer iteration in FP64. Also reported: the 64-mesh batched
workload, and the per-kernel figures on the 128^3 quarter-annulus.
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

# HBM bytes per dense-solve launch (k_gemv_whole_f64) on the 64^3 workload from hardware counters
# (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, per dispatch, scaled by the same
# counters read on a 1 GiB device copy: FETCH x2.0, WRITE x1.0), and the
# fingerprint of the GEMV source they were taken on. A changed kernel reports
# traffic as unknown until the counters are taken again.
GEMV_TRAFFIC = {"bytes": 1142612987, "fetch_kib": 556422.89, "write_kib": 2987.22, "fetch_scale": 2.0,
                "write_scale": 1.0, "src": "0c72c6b9fc27f9aa"}


def _gemv_source_fingerprint():
    import hashlib
    path = os.path.join(ROOT, "paper_2606_20496_amd", "csrc", "kernels.hip")
    src = open(path).read()
    i = src.index("void k_gemv_f64(")
    a = src.rindex("\n// ----", 0, src.rindex("// ----", 0, i))
    b = src.index("__global__", i)
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def run_form(torch, coarse, mesh, rhs, precision, steps, warmup, tol):
    """Set up once, then time `steps` solves, each on its own right-hand side (all
    resident on the GPU). Only the dominant kernel is bracketed by HIP events in
    the timed region; a separate pass afterwards times every phase."""
    t0 = time.perf_counter()
    S = coarse.CoarseSolver.from_mesh(mesh, precision=precision)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
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
        "relres_true_max": worst, "setup_s": t_setup, "info": info,
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
            "gemv_avg_launch_us": round(avg_ms * 1e3, 2), "gemv_alg_bytes": lb,
            "gemv_achieved_GBs": round(lb / (avg_ms / 1e3) / 1e9, 1)}


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
    R_p+J^T stage 1: per packed entry index + r value + r_p write; per J entry
           vertex id, weight, 3 local coordinates and the r value
    sum+J: per packed entry position + z_p; per free vertex cover pointer, r read,
           z written, J pointer; per J entry base corner, weight, 3 coordinates
    x,r update: x, r read and written, p, q read per free vertex."""
    es = 8 if precision == "fp64" else 4
    nf, snp, nj = info["n_free"], info["sum_np"], info["n_jent"]
    return {
        "A+p": n_elem * (224 + 16) + nf * 32,
        "R_p+J^T": snp * (4 + 8 + es) + nj * (4 + es + 3 * es + 8),
        "sum+J": snp * (4 + 8) + nf * (4 + 8 + 8 + 4) + nj * (4 + es + 3 * es),
        "x,r update": nf * 48,
    }


def run_kernels_large(torch, coarse, mg, tol):
    """The operator and interpolation kernels on the 128^3 quarter-annulus (2.1M
    elements, 4096 subdomains), where launch latency is amortised: HIP-event
    timings of every launch over one whole solve, against algorithmic bytes."""
    mesh = mg.large_annulus()
    out = {"workload": "annulus128: 128^3 quarter-annulus, radial ratio 1.05, 4096 subdomains of 8^3, "
                       "16^3 boxes", "n_elem": mesh.n_elem}
    b = torch.tensor(mesh.b, device="cuda")
    u = torch.empty_like(b)
    for prec in ("fp64", "mixed", "mixed16"):
        t0 = time.perf_counter()
        S = coarse.CoarseSolver.from_mesh(mesh, precision=prec)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        S.solve(b, tol, out=u)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, st = S.solve(b, tol, out=u)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t1
        S.profile_start(0xFF)
        S.solve(b, tol, out=u)
        ph = S.profile_stop()
        info = dict(S.info)
        S.close()
        kb = kernel_bytes(info, mesh.n_elem, prec)
        ks = {}
        for name, (ms, cnt) in ph.items():
            avg = ms / max(cnt, 1) * 1e3
            e = {"avg_us": round(avg, 2), "launches": cnt}
            if name in kb and avg > 0:
                gbs = kb[name] / (avg * 1e-6) / 1e9
                e.update(alg_bytes=kb[name], GBs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))
            ks[name] = e
        gm = ph[coarse.PHASES[GEMV_PHASE]]
        gavg = gm[0] / max(st["iters"], 1) * 1e3
        lb = local_inv_bytes(info, prec)
        ks[coarse.PHASES[GEMV_PHASE]].update(
            alg_bytes=lb, avg_us_work=round(gavg, 2), GBs=round(lb / (gavg * 1e-6) / 1e9, 1),
            frac=round(lb / (gavg * 1e-6) / 1e9 / HBM_PEAK_GBS, 4))
        out[prec] = {"iters": st["iters"], "relres_true": st["relres_true"], "solve_ms": round(1e3 * t_solve, 3),
                     "solves_per_s": round(1.0 / t_solve, 3), "setup_s": round(t_setup, 3), "kernels": ks}
        _log(f"annulus128 {prec}: {st['iters']} iters, {1e3 * t_solve:.2f} ms/solve")
    return out


def run_ablations(torch, coarse, mesh, b, tol, max_it=400):
    """Iterations to the tolerance for the preconditioner's parts and variants on
    the bench mesh (FP64): the additive two-level method, its local part alone,
    its reduced part alone, the symmetrised coarse-local-coarse hybrid, and two
    layers of overlap (the paper's study of the parts, Sec. 5)."""
    out = {}
    for name, kw in (("additive", {}), ("local_only", {"mode": "local_only"}),
                     ("reduced_only", {"mode": "reduced_only"}), ("hybrid_sym", {"mode": "hybrid_sym"}),
                     ("additive_overlap2", {"overlap": 2})):
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


def cpu_baseline(mesh, tol):
    """The FP64 oracle, as it stands, on the host cores: one full solve of the
    same workload (setup timed separately and excluded)."""
    cores = len(os.sched_getaffinity(0))
    from oracle import problem
    t0 = time.perf_counter()
    P = problem.from_mesh(mesh)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    u, info = P.solve(mesh.b, tol=tol)
    t = time.perf_counter() - t0
    return {"value": 1.0 / t, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"one full FP64 PCG solve of the 64^3 workload (first RHS) ({info['iters']} iterations, "
                      f"{t:.1f} s; oracle setup {t_setup:.1f} s excluded)",
            "iters": info["iters"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--n", type=int, default=64, help="cube edge in elements (64 = one GPU's share)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-mesh batched workload")
    ap.add_argument("--no-large", action="store_true", help="skip the 128^3 annulus kernel measurements")
    ap.add_argument("--no-ablations", action="store_true", help="skip the preconditioner-part study")
    ap.add_argument("--no-warm-start", action="store_true", help="skip the successive right-hand-side study")
    ap.add_argument("--no-multi", action="store_true", help="skip the 16-right-hand-side block solve")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the open-loop serving study over resident contexts")
    ap.add_argument("--serving", action="store_true", help="also run a short serving-loop workload")
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
    mesh = mg.gpu_share_cube(n=args.n)
    nrhs = min(args.steps + args.warmup, 32)
    rhs = [torch.tensor(mesh.b if i == 0 else mg.rhs_bumps(mesh, 100 + i), device="cuda") for i in range(nrhs)]

    _log("fp64 form")
    fp64 = run_form(torch, coarse, mesh, rhs, "fp64", args.steps, args.warmup, args.tol)
    _log(f"fp64: {fp64['solves_per_s']:.2f} solves/s")
    mixed = mixed16 = None
    if not args.no_mixed:
        mixed = run_form(torch, coarse, mesh, rhs, "mixed", args.steps, args.warmup, args.tol)
        _log(f"mixed: {mixed['solves_per_s']:.2f} solves/s")
        mixed16 = run_form(torch, coarse, mesh, rhs, "mixed16", args.steps, args.warmup, args.tol)
        _log(f"mixed16: {mixed16['solves_per_s']:.2f} solves/s")

    # roofline of the dominant kernel: the batched dense solve of the local systems
    # (tiled symmetric GEMV over their stored inverses), HBM-bound
    ms, cnt = fp64["gemv"]
    avg_s = ms / max(fp64["gemv_work_launches"], 1) / 1e3
    alg_bytes = local_inv_bytes(fp64["info"], "fp64")
    achieved = alg_bytes / avg_s / 1e9 if avg_s > 0 else 0.0
    traffic = GEMV_TRAFFIC["bytes"] if (args.n == 64 and _gemv_source_fingerprint() == GEMV_TRAFFIC["src"]) else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_gemv_whole_f64", "avg_launch_us": round(avg_s * 1e6, 2),
            "launches": cnt, "work_launches": fp64["gemv_work_launches"],
            "alg_bytes_per_launch": alg_bytes}
    phases = {k: {"avg_us": round(1e3 * v[0] / max(v[1], 1), 2), "launches": v[1]} for k, v in fp64["phases"].items()}

    batch = None
    if not args.no_batch:
        _log("batch workload")
        batch = run_batch_workload(torch, coarse, mg, args.tol)
        _log(f"batch: {batch}")
    ablations = None
    if not args.no_ablations:
        _log("ablations")
        ablations = run_ablations(torch, coarse, mesh, rhs[0], args.tol)
        _log(f"ablations: { {k: v['iters'] for k, v in ablations.items()} }")

    resident = None
    if not args.no_serving:
        _log("serving over resident contexts")
        resident = run_serving_resident(torch, coarse, mg, args.tol)

    warm = None
    if not args.no_warm_start:
        _log("warm start")
        warm = run_warm_start(torch, coarse, mg, mesh, args.tol)
        _log(f"warm start: {warm}")

    multi = None
    if not args.no_multi:
        _log("block solve, 16 right-hand sides")
        multi = run_multi(torch, coarse, mg, mesh, args.tol, max(2, args.steps // 4), 1)
        multi["vs_single_fp64"] = round(multi["solves_per_s"] / fp64["solves_per_s"], 2)
        if mixed16 is not None:
            m16 = run_multi(torch, coarse, mg, mesh, args.tol, max(2, args.steps // 4), 1, precision="mixed16")
            m16["vs_single_mixed16"] = round(m16["solves_per_s"] / mixed16["solves_per_s"], 2)
            multi["mixed16"] = m16
        _log(f"block solve: {multi}")

    large = None
    if not args.no_large:
        _log("annulus128 kernels")
        large = run_kernels_large(torch, coarse, mg, args.tol)

    serving = None
    if args.serving:
        # the full-size serving workload once ended in a host segmentation fault
        # whose cause has not been found; it stays switched off until it is
        print("--serving is disabled: a full-size serving run crashed (host segmentation fault) "
              "and the cause has not been found", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not args.no_cpu_baseline:
        _log("cpu baseline (oracle)")
        cpu = cpu_baseline(mesh, args.tol)

    line = {
        "metric": "coarse solves/sec to 1e-8 rel. residual (mixed vs FP64); p50/p99 latency",
        "value": round(fp64["solves_per_s"], 3),
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
        "config": {"workload": f"cube{args.n}: {args.n}^3 jittered Q1 hex cube, randomly renumbered, "
                               f"Dirichlet x=0; {mesh.n_part} subdomains of 8^3 elements, overlap 1; "
                               f"{mesh.boxes[0]}^3 boxes; PCG to {args.tol:g}",
                   "n_elem": mesh.n_elem, "n_free": mesh.n_free, "n_sub": fp64["info"]["n_sub"],
                   "n_r": fp64["info"]["n_r"]},
        "p50_ms": round(fp64["p50_ms"], 4),
        "p99_ms": round(fp64["p99_ms"], 4),
        "iters": fp64["iters"],
        "iters_range": [fp64["iters_min"], fp64["iters_max"]],
        "relres_true_max": fp64["relres_true_max"],
        "setup_s": round(fp64["setup_s"], 3),
        "mixed": _form_summary(mixed, "f32 local/reduced inverses, f32 J, f64 operator/vectors/dots", "mixed"),
        "mixed16": _form_summary(mixed16, "f16 storage of the local/reduced inverses (power-of-two scale per "
                                          "system), f32 arithmetic, f32 J, f64 operator/vectors/dots", "mixed16"),
        "phases_fp64": phases,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if batch is not None:
        line["batch_workload"] = batch
    if large is not None:
        line["large_workload"] = large
    if ablations is not None:
        line["ablations"] = ablations
    if warm is not None:
        line["warm_start"] = warm
    if multi is not None:
        line["multi_rhs"] = multi
    if resident is not None:
        line["serving_resident"] = resident
    if serving is not None:
        line["serving_workload"] = serving
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
