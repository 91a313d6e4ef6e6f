"""Write tests/golden/c3_oracle.json: the FP64 oracle's solve of the 128^3
quarter-annulus workload (2.1M elements, 4096 subdomains of 8^3 elements, 16^3
boxes, radial ratio 1.05; Dirichlet on r = 1, right-hand side i.i.d. N(0,1)).

Calls only the oracle and the seeded mesh generator. The oracle runs PCG from
x0 = 0 with the additive two-level Schwarz preconditioner of eq. (asm) and the
Fletcher-Reeves beta until ||r||_2 <= 1e-8 ||b||_2 (free entries). Recorded:
the iteration count, the recurrence residual after every iteration, the true
residual, norms of u, u at 64 seeded free vertices (user ids), the Lanczos
estimate of the extreme eigenvalues of M^{-1}A from the CG coefficients, and the
oracle's wall times with the host it ran on.

    python tests/golden/make_c3_oracle.py          (about 10 minutes, ~30 GB)
"""
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import pcg, problem  # noqa: E402
from paper_2606_20496_amd import meshgen as mg  # noqa: E402

N_SAMPLES = 64
SAMPLE_SEED = 31


def host_info():
    model = platform.processor() or ""
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
        cfg = np.show_config(mode="dicts")
        b = cfg["Build Dependencies"]["blas"]
        blas = f"{b.get('name', '?')} {b.get('version', '')}".strip()
    except Exception:  # noqa: BLE001
        pass
    return {"cores": len(os.sched_getaffinity(0)), "cpu_model": model, "blas": blas,
            "numpy": np.__version__}


def main(out=os.path.join(HERE, "c3_oracle.json")):
    t0 = time.perf_counter()
    m = mg.large_annulus()
    t_mesh = time.perf_counter() - t0
    print(f"mesh: {m.n_elem} elements, {m.n_vert} vertices ({t_mesh:.1f} s)", flush=True)
    t0 = time.perf_counter()
    P = problem.from_mesh(m)
    t_setup = time.perf_counter() - t0
    print(f"oracle setup {t_setup:.1f} s; n_free {P.A.shape[0]}, n_r {P.coarse.n_r}", flush=True)
    t0 = time.perf_counter()
    u, info = P.solve(m.b, tol=1e-8, record=True)
    t_solve = time.perf_counter() - t0
    print(f"oracle solve {t_solve:.1f} s, {info['iters']} iterations, relres {info['relres']:.3e}, "
          f"true {info['relres_true']:.3e}", flush=True)
    lo, hi = pcg.lanczos_condition(info["alphas"], info["betas"])
    free = np.flatnonzero(~m.dirichlet.astype(bool))
    ids = np.sort(np.random.default_rng(SAMPLE_SEED).choice(free, N_SAMPLES, replace=False))
    uf = u[free]
    rec = {
        "workload": "annulus128: 128^3 quarter annulus r in [1,2], theta in [0,pi/2], z in [0,1], "
                    "radial ratio 1.05, jitter 0.05 of the local spacing, seed 3; Dirichlet r=1; "
                    "b ~ N(0,1); 4096 subdomains of 8^3 elements, overlap 1; 16^3 boxes",
        "method": "PCG from x0=0, additive two-level Schwarz eq. (asm), Fletcher-Reeves beta, "
                  "stop at ||r||_2 <= 1e-8 ||b||_2 (recurrence residual, free entries)",
        "n_elem": m.n_elem, "n_vert": m.n_vert, "n_free": int(free.size),
        "n_sub": int(m.n_part), "n_r": int(P.coarse.n_r),
        "tol": 1e-8,
        "iters": int(info["iters"]),
        "relres": float(info["relres"]),
        "relres_true": float(info["relres_true"]),
        "relres_hist": [float(x) for x in info["relres_hist"]],
        "u_norm2": float(np.linalg.norm(uf)),
        "u_norminf": float(np.abs(uf).max()),
        "b_norm2": float(np.linalg.norm(m.b[free])),
        "sample_seed": SAMPLE_SEED,
        "sample_ids": [int(i) for i in ids],
        "u_samples": [float(u[i]) for i in ids],
        "lanczos_lambda_min": lo, "lanczos_lambda_max": hi,
        "oracle_setup_s": round(t_setup, 2),
        "oracle_solve_s": round(t_solve, 2),
        "oracle_s_per_iter": round(t_solve / max(1, info["iters"]), 4),
        "host": host_info(),
        "script": "tests/golden/make_c3_oracle.py",
    }
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main()
