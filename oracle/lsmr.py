"""LSMR (Fong & Saunders, 2011) for min ||A x - b||, optionally right-preconditioned by a
column scaling d: the iteration runs on A diag(d) and returns diag(d) times its iterate,
which leaves the residual unchanged.

Test infrastructure: this module is imported only by the tests, the smoke check and the
CPU baseline of the benchmark.

The paper solves both least-squares problems of the derivative with LSMR, the Krylov method
that needs only products with F and F' (Sec. 3.1, "Computing the derivative"; Sec. 3.2,
"Computing the adjoint"). LSMR builds the same Golub-Kahan bidiagonalisation as LSQR,
    beta_1 u_1 = b,  alpha_1 v_1 = A' u_1,
    beta_{k+1} u_{k+1} = A v_k - alpha_k u_k,  alpha_{k+1} v_{k+1} = A' u_{k+1} - beta_{k+1} v_k,
but picks the iterate x_k in span(v_1..v_k) that minimises ||A' r_k||. With B_k the lower
bidiagonal matrix of the alphas and betas:
  * a QR factorisation of B_k (rotations c_k, s_k) gives the upper bidiagonal R_k with
    diagonal rho_k and superdiagonal theta_{k+1};
  * minimising ||A' r_k|| reduces to a least-squares problem in t = R_k y whose matrix is
    [R_k'; theta_{k+1} e_k'] (lower bidiagonal); a second QR (rotations cbar, sbar) gives
    R_bar_k (diagonal rhobar_k, superdiagonal thetabar_{k+1}) and the right-hand side
    (zeta_1 .. zeta_k, zetabar_{k+1});
  * x_k = V_k R_k^{-1} R_bar_k^{-1} z_k is updated with two direction vectors h, hbar.

Residual estimate, written out here from the same factorisations: r_k = U_{k+1}(beta_1 e_1
- B_k y_k), so ||r_k||^2 = ||betahat_{1:k} - t_k||^2 + betadd_k^2, where (betahat, betadd) is
beta_1 e_1 after the rotations of the first QR, and t_k solves R_bar_k t = z_k. A third QR,
of R_bar_k' (rotations ctil, stil: diagonal rhotil, superdiagonal thetatil, unfinished last
diagonal rhodot), turns the back substitution into a forward one, tau = R_til^{-T} z, whose
leading entries no longer change; applying the same rotations to betahat gives betatil
(fixed) and betadot (the unfinished last entry). Then
    ||r_k||^2 = sum_{i<k} (betatil_i - tautil_i)^2 + (betadot_k - taudot_k)^2 + betadd_k^2.

Stopping rule: the estimate of ||b - A x_k|| falls to tol * ||b|| (the same rule as the
LSQR oracle, and as SciPy's lsmr with atol = 0, btol = tol).
"""
from __future__ import annotations

import math

import numpy as np


def lsmr(matvec, rmatvec, b, tol=1e-8, max_iter=None, col_scale=None, trace=None):
    """Returns (x, info) with info = dict(iters, est_residual, converged). When `trace` is a
    list, the relative residual estimate of every iteration is appended to it."""
    b = np.asarray(b, dtype=np.float64)
    d = None if col_scale is None else np.asarray(col_scale, dtype=np.float64)

    def Av(v):
        return matvec(v * d) if d is not None else matvec(v)

    def ATu(u):
        return rmatvec(u) * d if d is not None else rmatvec(u)

    # bidiagonalisation start
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
        return x, dict(iters=0, est_residual=1.0, converged=True)
    v /= alpha
    beta1 = beta

    # first QR (of B_k): alphabar is the unfinished diagonal entry
    alphabar = alpha
    # second QR (of [R_k'; theta e_k']): previous rho, rhobar and rotation
    rho_prev, rhobar_prev, cbar, sbar = 1.0, 1.0, 1.0, 0.0
    zetabar = alpha * beta
    h = v.copy()
    hbar = np.zeros(ncols)
    # residual estimate: beta_1 e_1 under the first QR, then the third QR
    betadd = beta              # last entry of the rotated beta_1 e_1
    betadot = 0.0              # unfinished entry after the third QR
    rhodot = 1.0               # unfinished diagonal of the third QR
    thetatil = 0.0             # superdiagonal of the third QR from the previous step
    tautil_prev = 0.0          # tau entry k-2 (fixed)
    zeta_prev = 0.0            # zeta_{k-1}
    fixed_sq = 0.0             # sum over fixed entries of (betatil - tautil)^2

    it = 0
    converged = False
    est = 1.0
    while it < max_iter:
        it += 1
        u = Av(v) - alpha * u
        beta = float(np.linalg.norm(u))
        if beta > 0:
            u /= beta
        v = ATu(u) - beta * v
        alpha = float(np.linalg.norm(v))
        if alpha > 0:
            v /= alpha

        # first QR: rotation eliminating beta_{k+1} under alphabar_k
        rho = math.hypot(alphabar, beta)
        c, s = alphabar / rho, beta / rho
        theta_next = s * alpha
        alphabar = c * alpha

        # second QR: rotation eliminating theta_{k+1} under cbar_{k-1} rho_k
        thetabar = sbar * rho
        rhobar = math.hypot(cbar * rho, theta_next)
        cbar_new = cbar * rho / rhobar
        sbar = theta_next / rhobar
        cbar = cbar_new
        zeta = cbar * zetabar
        zetabar = -sbar * zetabar

        # iterate and directions
        hbar = h - (thetabar * rho / (rho_prev * rhobar_prev)) * hbar
        x = x + (zeta / (rho * rhobar)) * hbar
        h = v - (theta_next / rho) * h
        rho_prev, rhobar_prev = rho, rhobar

        # residual estimate: first-QR rotation of (betadd, 0)
        betahat = c * betadd
        betadd = -s * betadd
        # third QR: rotation eliminating thetabar_k under rhodot_{k-1}; it fixes entry k-1
        rhotil = math.hypot(rhodot, thetabar)
        ctil, stil = rhodot / rhotil, thetabar / rhotil
        thetatil_new = stil * rhobar
        rhodot = ctil * rhobar
        betatil = ctil * betadot + stil * betahat
        betadot = -stil * betadot + ctil * betahat
        if it > 1:
            tautil = (zeta_prev - thetatil * tautil_prev) / rhotil
            fixed_sq += (betatil - tautil) ** 2
            tautil_prev = tautil
        thetatil = thetatil_new
        taudot = (zeta - thetatil * tautil_prev) / rhodot
        zeta_prev = zeta
        est = math.sqrt(fixed_sq + (betadot - taudot) ** 2 + betadd ** 2) / beta1
        if trace is not None:
            trace.append(est)
        if est <= tol or alpha == 0.0:
            converged = True
            break
    if d is not None:
        x = x * d
    return x, dict(iters=it, est_residual=est, converged=converged)
