"""Autotuner for the batched dense solve.

Two choices are tuned per precision, by timing the dense-solve launches (with
the partial-sum pass of the work items) on synthetic meshes:

* Tiles per work item, per size bucket of a system's tile count. A context with
  fewer systems than the device has compute units (every batch and serving mesh)
  cuts all its systems into work items, each a run of 32 x 32 tiles of one tile
  row that one wavefront streams; so do larger contexts for systems above 48 tile
  rows. The item length trades the per-item start-up (work-table loads,
  row-partial write) against load balance and column-partial traffic. Buckets
  0-6 are timed on meshes of 125 subdomains (every system an item), bucket 7 on
  a mesh of large systems.
* Wavefronts per workgroup for the systems of 16-48 tile rows that contexts with
  at least one system per compute unit solve one workgroup each (timed on the
  64^3 cube's 512 systems of 23 tile rows).

The fastest choices go to ``gemv_tuning.json`` next to this file (or ``--out``),
which ``coarse.gemv_table`` and ``coarse.whole_waves_choice`` read for every new
context. Run on the GPU: ``python -m paper_2606_20496_amd.tune [--out PATH]``.
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
ITEM_BUCKETS = tuple(range(8))
SMALL_K = 5            # 5^3 = 125 subdomains: fewer systems than compute units
WAVE_CANDIDATES = {"fp64": (2, 4, 8), "mixed": (4, 8, 16), "mixed16": (4, 8, 16)}
TILE_BYTES = {"fp64": 8, "mixed": 4, "mixed16": 2}
GEMV_PHASE = 3


def _log(msg):
    print(f"[tune] {msg}", file=sys.stderr, flush=True)


def _mesh_for(bucket, precision, target_bytes):
    """A mesh whose interior subdomain systems fall in `bucket`: 125 subdomains
    for the buckets the batch and serving meshes use, larger meshes of big
    systems for the last bucket."""
    block = BUCKET_BLOCK[bucket]
    n_p = (block + 1) ** 3
    nb = math.ceil(n_p / 32)
    k = SMALL_K
    if bucket == len(BUCKET_BLOCK) - 1:
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
    used = S.info["whole_waves"]
    S.close()
    # the dense-solve launch and, when work items were used, their partial sums
    ms, cnt = ph[coarse.PHASES[GEMV_PHASE]]
    ms_c, _ = ph[coarse.PHASES[GEMV_PHASE + 1]]
    return 1e3 * (ms + ms_c) / max(cnt, 1), used


def tune(precision, target_bytes=1.0e9, reps=20):
    import torch
    table = [4] * coarse.GEMV_BUCKETS
    timings = {}
    for b in ITEM_BUCKETS:
        t0 = time.perf_counter()
        m, nb = _mesh_for(b, precision, target_bytes)
        plan = coarse.Plan.from_mesh(m, precision=precision)
        res = {}
        for c in CANDIDATES:
            if c > nb and res:
                break
            tiles = [4] * coarse.GEMV_BUCKETS
            tiles[b] = c
            res[c] = round(time_gemv(torch, plan, m.n_vert, tiles, reps)[0], 2)
        plan.close()
        best = min(res, key=res.get)
        table[b] = best
        timings[str(b)] = {"block": BUCKET_BLOCK[b], "nb": nb, "n_elem": m.n_elem, "n_sub": m.n_part, "us": res}
        _log(f"{precision} bucket {b} (nb {nb}, {m.n_part} systems): {res} -> {best} "
             f"({time.perf_counter() - t0:.1f} s)")
    # wavefronts per whole-system workgroup, on the 64^3 cube (512 systems of 23 tile rows)
    m = mg.gpu_share_cube()
    waves = {}
    for w in WAVE_CANDIDATES[precision]:
        plan = coarse.Plan.from_mesh(m, precision=precision, whole_waves=w)
        us, used = time_gemv(torch, plan, m.n_vert, table, reps)
        plan.close()
        if used == w:
            waves[w] = round(us, 2)
    best_w = min(waves, key=waves.get)
    _log(f"{precision} whole-system wavefronts: {waves} -> {best_w}")
    return table, best_w, timings, waves


def main():
    ap = argparse.ArgumentParser(description="tune the dense-solve work items and whole-system workgroups")
    ap.add_argument("--out", default=coarse.TUNING_PATH)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--bytes", type=float, default=1.0e9, help="stored inverse bytes of the large-system mesh")
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        sys.exit("the tuner times GPU kernels; no GPU is available")
    coarse.load()
    out = {"device": torch.cuda.get_device_name(0),
           "arch": getattr(torch.cuda.get_device_properties(0), "gcnArchName", ""),
           "bucket_max": list(coarse.GEMV_BUCKET_MAX), "candidates": list(CANDIDATES)}
    for prec in PRECISIONS:
        table, w, timings, waves = tune(prec, args.bytes, args.reps)
        out[prec] = {"tiles_per_item": table, "whole_waves": w, "timings_us": timings,
                     "whole_waves_us": {str(k): v for k, v in waves.items()}}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({p: [out[p]["tiles_per_item"], out[p]["whole_waves"]] for p in PRECISIONS}), flush=True)


if __name__ == "__main__":
    main()
