"""Derivative (JVP) and adjoint (VJP) of the QCP solution map.

jvp / vjp           -- the paper's steps (Sec. 3.1 and 3.2): z = (x, y - s, 1); the JVP solves
                       min ||F dz + D_theta N[dtheta]|| and maps dz through D phi; the VJP maps
                       the cotangent through D phi', solves min ||F' w + dz||, and returns
                       D_theta N'[w] restricted to the stored patterns of P and A. The
                       least-squares solver is LSQR or LSMR (the paper's), both matrix-free.
jvp_dense/vjp_dense -- the implicit function theorem applied to the KKT conditions in Minty
                       form with tau fixed to 1 (Sec. 2.3, eq. minty-restrictions is equivalent
                       to eq. kkt-conds):
                           G(xi, eta; theta) = (P xi + A' Pi(eta) + q, -A xi + b - Pi(eta) + eta)
                       with (x, y, s) = (xi, Pi(eta), Pi(eta) - eta). Its Jacobian in (xi, eta)
                       is K_red = [[P, A'J], [-A, I - J]], J = DPi_{K*}(eta). Dense LU solves.
qp_active_set_jvp   -- the textbook derivative of a QP's solution with a fixed active set
                       (zero and nonnegative cones only).
newton_resolve      -- a semismooth Newton solve of G(.; theta') = 0, used to take finite
                       differences of the solution map through values only.

Reading: F is singular (F z = 0 by positive homogeneity of R, Sec. 2.3), so the least
squares problems are consistent but have a one-dimensional null space; any least-squares
solution gives the same (dx, dy, ds) and dtheta, which is what is compared.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import cones as C
from .embedding import Embedding, _coords
from .lsmr import lsmr
from .lsqr import lsqr

_SOLVERS = {"lsqr": lsqr, "lsmr": lsmr}


# ----------------------------------------------------------------------------------------
# Jacobi column scaling (right preconditioning): 1 / column norms of F with each cone-block
# Jacobian replaced by its diagonal.
# ----------------------------------------------------------------------------------------

def _sq_rows(M):
    return np.asarray(M.multiply(M).sum(axis=1)).ravel()


def _sq_cols(M):
    return np.asarray(M.multiply(M).sum(axis=0)).ravel()


def jacobi_scale_F(emb: Embedding):
    q = emb.qcp
    jd = emb.J.diagonal()
    c = -2.0 * emb.Px - q.q
    colx = _sq_cols(q.P) + _sq_cols(q.A) + c * c
    coly = jd * jd * (_sq_rows(q.A) + q.b * q.b) + (1.0 - jd) ** 2
    colN = q.q @ q.q + q.b @ q.b + emb.xPx ** 2
    nrm = np.sqrt(np.concatenate([colx, coly, [colN]]))
    return np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1.0), 1.0)


def jacobi_scale_FT(emb: Embedding):
    """Row norms of F (= column norms of F') with the same diagonal approximation."""
    q = emb.qcp
    jd = emb.J.diagonal()
    c = -2.0 * emb.Px - q.q
    AJ = q.A.multiply(jd[:, None]) if q.m else q.A
    rowx = _sq_rows(q.P) + _sq_cols(AJ) + q.q * q.q
    rowy = _sq_rows(q.A) + (1.0 - jd) ** 2 + q.b * q.b
    rowN = c @ c + (q.b * jd) @ (q.b * jd) + emb.xPx ** 2
    nrm = np.sqrt(np.concatenate([rowx, rowy, [rowN]]))
    return np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1.0), 1.0)


# ----------------------------------------------------------------------------------------
# the paper's method (Sec. 3.1, 3.2)
# ----------------------------------------------------------------------------------------

def jvp(qcp, dP, dA, dq, db, tol=None, max_iter=None, precond="jacobi", emb=None,
        return_info=False, solver="lsqr"):
    emb = emb or Embedding(qcp)
    tol = qcp.tol if tol is None else tol
    d = emb.dtheta(dP, dA, dq, db)
    scale = jacobi_scale_F(emb) if precond == "jacobi" else None
    dz, info = _SOLVERS[solver](emb.F, emb.FT, -d, tol=tol, max_iter=max_iter, col_scale=scale)
    dx, dy, ds = emb.dphi(dz)
    if return_info:
        bn = np.linalg.norm(d)
        info["rel_residual"] = float(np.linalg.norm(emb.F(dz) + d) / bn) if bn > 0 else 0.0
        return dx, dy, ds, info
    return dx, dy, ds


def vjp(qcp, gx, gy, gs, tol=None, max_iter=None, precond="jacobi", emb=None,
        return_info=False, solver="lsqr"):
    emb = emb or Embedding(qcp)
    tol = qcp.tol if tol is None else tol
    dz = emb.dphi_t(gx, gy, gs)
    scale = jacobi_scale_FT(emb) if precond == "jacobi" else None
    w, info = _SOLVERS[solver](emb.FT, emb.F, -dz, tol=tol, max_iter=max_iter, col_scale=scale)
    out = emb.dtheta_t(w)
    if return_info:
        bn = np.linalg.norm(dz)
        info["rel_residual"] = float(np.linalg.norm(emb.FT(w) + dz) / bn) if bn > 0 else 0.0
        return (*out, info)
    return out


# ----------------------------------------------------------------------------------------
# dense implicit-function-theorem reference on the reduced KKT matrix
# ----------------------------------------------------------------------------------------

def K_red(qcp, J_dense):
    P = qcp.P.toarray()
    A = qcp.A.toarray()
    m = qcp.m
    return np.block([[P, A.T @ J_dense], [-A, np.eye(m) - J_dense]])


def jvp_dense(qcp, dP, dA, dq, db):
    eta = qcp.y - qcp.s
    J = C.DualJacobian(eta, qcp.cones).dense_matrix()
    K = K_red(qcp, J)
    dPm = qcp.P.copy()
    dPm.data = np.asarray(dP, dtype=np.float64).copy()
    dAm = qcp.A.copy()
    dAm.data = np.asarray(dA, dtype=np.float64).copy()
    rhs = -np.concatenate([dPm @ qcp.x + dAm.T @ qcp.y + dq, -(dAm @ qcp.x) + db])
    sol = sla.solve(K, rhs)
    xi, et = sol[:qcp.n], sol[qcp.n:]
    Je = J @ et
    return xi, Je, Je - et


def vjp_dense(qcp, gx, gy, gs):
    eta = qcp.y - qcp.s
    J = C.DualJacobian(eta, qcp.cones).dense_matrix()
    K = K_red(qcp, J)
    lam = sla.solve(K.T, np.concatenate([gx, J @ (gy + gs) - gs]))
    lx, ly = lam[:qcp.n], lam[qcp.n:]
    Pi, Pj = _coords(qcp.P)
    Ai, Aj = _coords(qcp.A)
    x, y = qcp.x, qcp.y
    dP = -0.5 * (lx[Pi] * x[Pj] + x[Pi] * lx[Pj])
    dA = -(y[Ai] * lx[Aj] - ly[Ai] * x[Aj])
    return dP, dA, -lx, -ly


def jvp_vjp_dense(qcp, dP, dA, dq, db, gx, gy, gs):
    """jvp_dense and vjp_dense with one LU factorisation of K_red shared by both solves (the
    same definitions; for the larger instances, where the factorisation dominates). A' J is
    formed from the sparse A."""
    eta = qcp.y - qcp.s
    J = C.DualJacobian(eta, qcp.cones).dense_matrix()
    n, m = qcp.n, qcp.m
    K = np.empty((n + m, n + m))
    K[:n, :n] = qcp.P.toarray()
    K[:n, n:] = qcp.A.T @ J
    K[n:, :n] = -qcp.A.toarray()
    K[n:, n:] = np.eye(m) - J
    lu = sla.lu_factor(K, overwrite_a=True, check_finite=False)
    del K
    dPm = qcp.P.copy()
    dPm.data = np.asarray(dP, dtype=np.float64).copy()
    dAm = qcp.A.copy()
    dAm.data = np.asarray(dA, dtype=np.float64).copy()
    rhs = -np.concatenate([dPm @ qcp.x + dAm.T @ qcp.y + dq, -(dAm @ qcp.x) + db])
    sol = sla.lu_solve(lu, rhs, check_finite=False)
    xi, et = sol[:n], sol[n:]
    Je = J @ et
    lam = sla.lu_solve(lu, np.concatenate([gx, J @ (gy + gs) - gs]), trans=1, check_finite=False)
    lx, ly = lam[:n], lam[n:]
    Pi, Pj = _coords(qcp.P)
    Ai, Aj = _coords(qcp.A)
    x, y = qcp.x, qcp.y
    dPo = -0.5 * (lx[Pi] * x[Pj] + x[Pi] * lx[Pj])
    dAo = -(y[Ai] * lx[Aj] - ly[Ai] * x[Aj])
    return (xi, Je, Je - et), (dPo, dAo, -lx, -ly)


def kred_cond(qcp):
    eta = qcp.y - qcp.s
    J = C.DualJacobian(eta, qcp.cones).dense_matrix()
    return float(np.linalg.cond(K_red(qcp, J)))


# ----------------------------------------------------------------------------------------
# textbook QP derivative with a fixed active set (zero + nonnegative cones)
# ----------------------------------------------------------------------------------------

def qp_active_set_jvp(qcp, dP, dA, dq, db):
    assert not qcp.cones.soc and not qcp.cones.psd and not qcp.cones.n_exp
    nz = qcp.cones.n_zero
    act = np.concatenate([np.arange(nz), nz + np.nonzero(qcp.y[nz:] > 0)[0]])
    P = qcp.P.toarray()
    A = qcp.A.toarray()
    dPd = qcp.P.copy()
    dPd.data = np.asarray(dP, dtype=np.float64).copy()
    dPd = dPd.toarray()
    dAd = qcp.A.copy()
    dAd.data = np.asarray(dA, dtype=np.float64).copy()
    dAd = dAd.toarray()
    AH = A[act]
    h = act.size
    n = qcp.n
    KKT = np.block([[P, AH.T], [AH, np.zeros((h, h))]])
    rhs = np.concatenate([-(dPd @ qcp.x + dAd.T @ qcp.y + dq), db[act] - dAd[act] @ qcp.x])
    sol = sla.solve(KKT, rhs)
    dx = sol[:n]
    dy = np.zeros(qcp.m)
    dy[act] = sol[n:]
    ds = db - dAd @ qcp.x - A @ dx
    ds[act] = 0.0
    return dx, dy, ds


# ----------------------------------------------------------------------------------------
# semismooth Newton re-solve of G(xi, eta; theta) = 0 (values only define the root)
# ----------------------------------------------------------------------------------------

def G_map(qcp, xi, eta):
    py = C.proj_dual(eta, qcp.cones)
    return np.concatenate([qcp.P @ xi + qcp.A.T @ py + qcp.q,
                           -(qcp.A @ xi) + qcp.b - py + eta])


def newton_resolve(qcp, x0, eta0, tol=1e-14, max_iter=50):
    xi, eta = x0.copy(), eta0.copy()
    scale = 1.0 + np.linalg.norm(qcp.q) + np.linalg.norm(qcp.b)
    g = G_map(qcp, xi, eta)
    for _ in range(max_iter):
        if np.linalg.norm(g) <= tol * scale:
            break
        J = C.DualJacobian(eta, qcp.cones).dense_matrix()
        step = sla.solve(K_red(qcp, J), -g)
        xi = xi + step[:qcp.n]
        eta = eta + step[qcp.n:]
        g_new = G_map(qcp, xi, eta)
        if np.linalg.norm(g_new) >= np.linalg.norm(g) and np.linalg.norm(g_new) < 1e3 * tol * scale:
            g = g_new
            break
        g = g_new
    py = C.proj_dual(eta, qcp.cones)
    return xi, py, py - eta, float(np.linalg.norm(g) / scale)
