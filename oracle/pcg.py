"""Preconditioned conjugate gradients — oracle (test infrastructure).

The outer iteration of the coarse solve (Sec. 1 footnote: the coarse problem is
embedded in a Krylov method; here it is solved by PCG to a relative residual).
Standard PCG from x0 = 0: q = A p, alpha = (r,z)/(p,q), x += alpha p,
r -= alpha q, stop when ||r||_2 <= tol ||b||_2, z = M r,
beta = (r,z)_new / (r,z)_old (Fletcher-Reeves) or, when ``flexible``,
beta = (r_new, z_new - z_old) / (r,z)_old (Polak-Ribiere), p = z + beta p.
The iteration count is the number of products with A in the loop.
"""
from __future__ import annotations

import numpy as np


def pcg(matvec, precond, b, tol=1e-8, max_it=1000, flexible=False, record=False):
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = float(np.sqrt(b @ b))
    info = {"iters": 0, "relres": 0.0, "alphas": [], "betas": [], "relres_hist": [], "converged": True}
    if bnorm == 0.0:
        return x, info
    r = b.copy()
    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    it = 0
    relres = 1.0
    while it < max_it:
        q = matvec(p)
        pq = float(p @ q)
        if not (pq > 0.0) or not np.isfinite(pq):
            raise FloatingPointError("PCG breakdown: p.Ap <= 0")
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        relres = float(np.sqrt(r @ r)) / bnorm
        if record:
            info["alphas"].append(alpha)
            info["relres_hist"].append(relres)
        if relres <= tol:
            break
        znew = precond(r)
        rz_new = float(r @ znew)
        beta = (rz_new - float(r @ z)) / rz if flexible else rz_new / rz
        if record:
            info["betas"].append(beta)
        z = znew
        rz = rz_new
        p = z + beta * p
    info["iters"] = it
    info["relres"] = relres
    info["converged"] = relres <= tol
    return x, info


def lanczos_condition(alphas, betas):
    """Extreme eigenvalue estimates of M^{-1}A from the CG coefficients (the
    Lanczos tridiagonal T: T_jj = 1/a_j + b_{j-1}/a_{j-1}, T_j,j+1 = sqrt(b_j)/a_j)."""
    k = min(len(alphas), len(betas) + 1)
    if k == 0:
        return np.nan, np.nan
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])
