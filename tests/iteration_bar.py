"""The FP64 iteration-count bar against the oracle. The library must stop at
the oracle's own count, except where that count sits on a knife edge: the
residual crosses the tolerance within rounding, so that the oracle itself
stops one iteration earlier or later when b, or the output of its
preconditioner, is perturbed entrywise at 1e-13 (the library's explicit
inverses and the oracle's Cholesky solves differ at that level). There every
count the oracle reaches under those perturbations (four seeds each) is
correct. Oracle-only arithmetic; the perturbations are computed only when the
counts differ."""
import numpy as np


def oracle_counts(P, b, iters, tol=1e-8, flexible=False, seeds=4):
    """{iters} and the oracle's counts for b and its preconditioner perturbed."""
    b = np.asarray(b, dtype=np.float64)
    counts = {int(iters)}
    for seed in range(seeds):
        xi = np.random.default_rng(seed).standard_normal(b.shape[0])
        counts.add(P.solve(b * (1 + 1e-13 * xi), tol=tol, flexible=flexible)[1]["iters"])
    M0 = P.M
    try:
        for seed in range(seeds):
            xi = np.random.default_rng(100 + seed).standard_normal(P.A.shape[0])
            P.M = lambda v, xi=xi: M0(v) * (1 + 1e-13 * xi)
            counts.add(P.solve(b, tol=tol, flexible=flexible)[1]["iters"])
    finally:
        P.M = M0
    return counts


def check_fp64_iters(gpu_iters, P, b, iters, tol=1e-8, flexible=False, what=""):
    if int(gpu_iters) == int(iters):
        return
    counts = oracle_counts(P, b, iters, tol=tol, flexible=flexible)
    assert int(gpu_iters) in counts, (what, int(gpu_iters), sorted(counts))
