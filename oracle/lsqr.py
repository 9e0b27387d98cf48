"""LSQR (Paige & Saunders, 1982) for min ||A x - b||, optionally right-preconditioned by a
column scaling: A is replaced by A diag(d), and the returned x is diag(d) times the
iterate, which leaves the residual unchanged.

The paper solves its least-squares problems with a Krylov method that needs only products
with F and F' (Sec. 3.1, "we use LSMR ... which only requires multiplication with F and
F^T"); this oracle uses LSQR for both directions.

Stopping rule: the recurrence estimate of ||b - A x|| (phibar) falls to tol * ||b||, the
same first test as SciPy's lsqr with atol = 0, btol = tol.
"""
from __future__ import annotations

import math

import numpy as np


def lsqr(matvec, rmatvec, b, tol=1e-8, max_iter=None, col_scale=None):
    """Returns (x, info) with info = dict(iters, est_residual, converged)."""
    b = np.asarray(b, dtype=np.float64)
    ncols = None
    d = None if col_scale is None else np.asarray(col_scale, dtype=np.float64)

    def Av(v):
        return matvec(v * d) if d is not None else matvec(v)

    def ATu(u):
        return rmatvec(u) * d if d is not None else rmatvec(u)

    u = b.copy()
    beta = float(np.linalg.norm(u))
    if beta == 0.0:
        v = ATu(np.zeros_like(b))
        return np.zeros_like(v), dict(iters=0, est_residual=0.0, converged=True)
    u /= beta
    v = ATu(u)
    ncols = v.size
    if max_iter is None:
        max_iter = 20 * ncols
    alpha = float(np.linalg.norm(v))
    x = np.zeros(ncols)
    if alpha == 0.0:
        return x, dict(iters=0, est_residual=beta, converged=True)
    v /= alpha
    w = v.copy()
    phibar, rhobar = beta, alpha
    beta1 = beta
    it = 0
    converged = False
    while it < max_iter:
        it += 1
        # bidiagonalisation step
        u = Av(v) - alpha * u
        beta = float(np.linalg.norm(u))
        if beta > 0:
            u /= beta
        v = ATu(u) - beta * v
        alpha = float(np.linalg.norm(v))
        if alpha > 0:
            v /= alpha
        # plane rotation eliminating beta
        rho = math.hypot(rhobar, beta)
        c, s = rhobar / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        # update of the iterate and the search direction
        x = x + (phi / rho) * w
        w = v - (theta / rho) * w
        if phibar <= tol * beta1 or alpha == 0.0:
            converged = True
            break
    if d is not None:
        x = x * d
    return x, dict(iters=it, est_residual=phibar / beta1, converged=converged)
