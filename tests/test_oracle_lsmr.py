"""Pins for the oracle's LSMR (Fong & Saunders 2011; the paper's solver, Sec. 3.1-3.2).

* The iterate against SciPy's lsmr (library) on over- and under-determined systems, and
  least-squares optimality A'(b - Ax) = 0.
* The residual estimate of every iteration against the explicitly recomputed residual
  ||b - A x_k|| (brute force: the solve is rerun with max_iter = k), on consistent and
  inconsistent systems: a wrong rotation or index in the estimate's recurrences fails here.
* LSMR's defining property: ||A' r_k|| is non-increasing in k.
* Exact solutions of tiny nonsingular systems; the consistent singular system of the
  derivative (JVP of a mixed-cone instance) against the dense implicit-function solve.
* Planted mistakes in a copy of the recurrence fail the estimate pin.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import qcpgen
from oracle import derivative as D
from oracle import embedding as E
from oracle.lsmr import lsmr


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("shape", [(40, 25), (25, 40), (30, 30)])
def test_lsmr_matches_scipy(shape):
    rng = np.random.default_rng(shape[0] + 7)
    A = rng.standard_normal(shape)
    b = rng.standard_normal(shape[0])
    x, info = lsmr(lambda v: A @ v, lambda u: A.T @ u, b, tol=1e-14, max_iter=3000)
    ref = spla.lsmr(A, b, atol=0, btol=1e-14, maxiter=3000)[0]
    assert rel(x, ref) < 1e-9
    assert np.linalg.norm(A.T @ (b - A @ x)) < 1e-8 * np.linalg.norm(A) * np.linalg.norm(b)


@pytest.mark.parametrize("consistent", [True, False])
def test_residual_estimate_equals_explicit_residual(consistent):
    rng = np.random.default_rng(11 if consistent else 12)
    A = rng.standard_normal((24, 16)) @ np.diag(np.logspace(0, 2, 16))
    b = A @ rng.standard_normal(16) if consistent else rng.standard_normal(24)
    trace = []
    lsmr(lambda v: A @ v, lambda u: A.T @ u, b, tol=0.0, max_iter=14, trace=trace)
    nb = np.linalg.norm(b)
    for k in range(1, 15):
        xk, info = lsmr(lambda v: A @ v, lambda u: A.T @ u, b, tol=0.0, max_iter=k)
        explicit = np.linalg.norm(b - A @ xk) / nb
        assert info["iters"] == k
        assert abs(info["est_residual"] - explicit) <= 1e-10 * max(explicit, 1e-3), k
        assert trace[k - 1] == info["est_residual"]


def test_normal_residual_is_monotone():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((50, 30))
    b = rng.standard_normal(50)
    prev = math.inf
    for k in range(1, 30):
        xk, _ = lsmr(lambda v: A @ v, lambda u: A.T @ u, b, tol=0.0, max_iter=k)
        g = np.linalg.norm(A.T @ (b - A @ xk))
        assert g <= prev * (1 + 1e-12)
        prev = g


def test_lsmr_exact_on_nonsingular_and_scaled():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((12, 12)) + 4 * np.eye(12)
    xs = rng.standard_normal(12)
    b = A @ xs
    x, info = lsmr(lambda v: A @ v, lambda u: A.T @ u, b, tol=1e-15, max_iter=500)
    assert info["converged"] and rel(x, xs) < 1e-10
    d = rng.uniform(0.2, 5.0, 12)
    x2, _ = lsmr(lambda v: A @ v, lambda u: A.T @ u, b, tol=1e-15, max_iter=500, col_scale=d)
    assert rel(x2, xs) < 1e-10


def test_lsmr_zero_rhs():
    A = np.eye(3)
    x, info = lsmr(lambda v: A @ v, lambda u: A.T @ u, np.zeros(3))
    assert info["iters"] == 0 and not np.any(x)


def test_lsmr_jvp_of_mixed_instance_matches_dense():
    """The derivative's consistent singular system (F z = 0): LSMR's least-squares solution
    mapped through D phi equals the dense implicit-function solve."""
    q = qcpgen.small_mixed(0)
    emb = E.Embedding(q)
    d = emb.dtheta(q.dP, q.dA, q.dq, q.db)
    dz, info = lsmr(emb.F, emb.FT, -d, tol=1e-13, col_scale=D.jacobi_scale_F(emb))
    assert info["converged"]
    dx, dy, ds = emb.dphi(dz)
    ref = D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)
    for a, r in zip((dx, dy, ds), ref):
        assert rel(a, r) < 1e-9


def _estimate_with_mistake(A, b, iters, mistake):
    """A copy of the estimate's recurrence with one planted mistake, returning the final
    estimate (the iterate itself is not needed)."""
    u = b / np.linalg.norm(b)
    beta1 = np.linalg.norm(b)
    v = A.T @ u
    alpha = np.linalg.norm(v)
    v /= alpha
    alphabar, cbar, sbar, zetabar = alpha, 1.0, 0.0, alpha * beta1
    betadd, betadot, rhodot, thetatil, tautil_prev, zeta_prev, fixed = beta1, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0
    for it in range(1, iters + 1):
        u = A @ v - alpha * u
        beta = np.linalg.norm(u)
        u /= beta
        v = A.T @ u - beta * v
        alpha = np.linalg.norm(v)
        v /= alpha
        rho = math.hypot(alphabar, beta)
        c, s = alphabar / rho, beta / rho
        theta_next = s * alpha
        alphabar = c * alpha
        thetabar = sbar * rho
        rhobar = math.hypot(cbar * rho, theta_next)
        cbar = cbar * rho / rhobar
        sbar = theta_next / rhobar
        zeta = cbar * zetabar
        zetabar = -sbar * zetabar
        betahat = c * betadd
        betadd = -s * betadd
        rhotil = math.hypot(rhodot, thetabar)
        ctil, stil = rhodot / rhotil, thetabar / rhotil
        thetatil_new = stil * rhobar
        rhodot = ctil * rhobar
        betatil = ctil * betadot + stil * betahat
        betadot = -stil * betadot + ctil * betahat
        if it > 1:
            th = thetatil_new if mistake == "index" else thetatil
            tautil = (zeta_prev - th * tautil_prev) / rhotil
            fixed += (betatil - tautil) ** 2
            tautil_prev = tautil
        thetatil = thetatil_new
        taudot = (zeta - thetatil * tautil_prev) / rhodot
        zeta_prev = zeta
        betadd_term = 0.0 if mistake == "drop_betadd" else betadd ** 2
    return math.sqrt(fixed + (betadot - taudot) ** 2 + betadd_term) / beta1


@pytest.mark.parametrize("mistake", ["index", "drop_betadd"])
def test_planted_estimate_mistakes_fail(mistake):
    rng = np.random.default_rng(12)
    A = rng.standard_normal((24, 16)) @ np.diag(np.logspace(0, 2, 16))
    b = rng.standard_normal(24)
    k = 10
    xk, info = lsmr(lambda v: A @ v, lambda u: A.T @ u, b, tol=0.0, max_iter=k)
    explicit = np.linalg.norm(b - A @ xk) / np.linalg.norm(b)
    assert abs(_estimate_with_mistake(A, b, k, None) - explicit) <= 1e-10
    assert abs(_estimate_with_mistake(A, b, k, mistake) - explicit) > 1e-6
