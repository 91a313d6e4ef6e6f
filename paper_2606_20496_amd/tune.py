"""Autotuner for the batched dense solve.

Systems of up to 48 tile rows are solved by one workgroup each. Larger systems
(and the few smallest ones left over beyond a multiple of the compute-unit
count) are split into work items, each a run of 32 x 32 tiles of one tile row
that one wavefront streams. How many tiles an item holds trades the per-item
start-up (work-table loads, row-partial write) against load balance and the
column-partial traffic. This script times the dense-solve launches for every
candidate item length on synthetic meshes whose subdomain systems fall in the
tuned size buckets (those of ``coarse.GEMV_BUCKET_MAX`` above 48 tile rows),
for every precision, and writes the fastest choice per bucket to
``gemv_tuning.json`` next to this file (or to ``--out``), keeping the earlier
entries of the other buckets. ``coarse.gemv_table`` reads that file for every
new context.

Run on the GPU: ``python -m paper_2606_20496_amd.tune [--out PATH]``.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

from . import coarse, meshgen as mg

# Subdomain block (elements per side) whose interior systems, (block + 1)^3
# unknowns, land in each bucket: nb = 2, 4, 7, 11, 16, 23, 42, 69 tiles.
BUCKET_BLOCK = (3, 4, 5, 6, 7, 8, 10, 12)
CANDIDATES = (1, 2, 3, 4, 6, 8, 12, 16)
PRECISIONS = ("fp64", "mixed", "mixed16")
TUNED_BUCKETS = (7,)   # systems above 48 tile rows: the ones cut into work items
TILE_BYTES = {"fp64": 8, "mixed": 4, "mixed16": 2}
GEMV_PHASE = 3


def _log(msg):
    print(f"[tune] {msg}", file=sys.stderr, flush=True)


def _mesh_for(block, precision, target_bytes):
    n_p = (block + 1) ** 3
    nb = math.ceil(n_p / 32)
    es = TILE_BYTES[precision]
    sys_bytes = nb * (nb + 1) // 2 * 32 * 32 * es
    k = max(2, min(int(round((target_bytes / sys_bytes) ** (1 / 3))), 100 // block))
    return mg.box_mesh(block * k, 7000 + block, block=block, boxes=(k, k, k), name=f"tune{block}"), nb


def time_gemv(torch, plan, n_vert, tiles, reps):
    plan.set_gemv_tiles(tiles)
    S = coarse.CoarseSolver.from_plan(plan)
    r = torch.randn(n_vert, dtype=torch.float64, device="cuda")
    for _ in range(3):
        S.apply_precond(r)
    torch.cuda.synchronize()
    S.profile_start((1 << GEMV_PHASE) | (1 << (GEMV_PHASE + 1)))
    for _ in range(reps):
        S.apply_precond(r)
    ph = S.profile_stop()
    S.close()
    # the dense-solve launch and, when work items were used, their partial sums
    ms, cnt = ph[coarse.PHASES[GEMV_PHASE]]
    ms_c, _ = ph[coarse.PHASES[GEMV_PHASE + 1]]
    return 1e3 * (ms + ms_c) / max(cnt, 1)


def tune(precision, target_bytes=1.0e9, reps=20, previous=None):
    import torch
    table = list(previous) if previous else [4] * coarse.GEMV_BUCKETS
    timings = {}
    for b, block in enumerate(BUCKET_BLOCK):
        if b not in TUNED_BUCKETS:
            continue
        t0 = time.perf_counter()
        m, nb = _mesh_for(block, precision, target_bytes)
        plan = coarse.Plan.from_mesh(m, precision=precision)
        res = {}
        for c in CANDIDATES:
            if c > nb and res:
                break
            tiles = [4] * coarse.GEMV_BUCKETS
            tiles[b] = c
            res[c] = round(time_gemv(torch, plan, m.n_vert, tiles, reps), 2)
        plan.close()
        best = min(res, key=res.get)
        table[b] = best
        timings[str(b)] = {"block": block, "nb": nb, "n_elem": m.n_elem, "us": res}
        _log(f"{precision} bucket {b} (nb {nb}, {m.n_elem} elements): {res} -> {best} "
             f"({time.perf_counter() - t0:.1f} s)")
    return table, timings


def main():
    ap = argparse.ArgumentParser(description="tune the GEMV work-item length per size bucket")
    ap.add_argument("--out", default=coarse.TUNING_PATH)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--bytes", type=float, default=1.0e9, help="stored inverse bytes per tuning mesh")
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        sys.exit("the tuner times GPU kernels; no GPU is available")
    coarse.load()
    out = {"device": torch.cuda.get_device_name(0), "bucket_max": list(coarse.GEMV_BUCKET_MAX),
           "candidates": list(CANDIDATES)}
    for prec in PRECISIONS:
        table, timings = tune(prec, args.bytes, args.reps, previous=coarse.gemv_table(prec))
        out[prec] = {"tiles_per_item": table, "timings_us": timings}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({p: out[p]["tiles_per_item"] for p in PRECISIONS}), flush=True)


if __name__ == "__main__":
    main()
