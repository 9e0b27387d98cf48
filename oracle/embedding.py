"""The homogeneous-embedding algebra of Sec. 2 written out on a QCP instance.

Notation (Sec. 2.1, eq. embedding): N = n + m + 1, u = (x, y, tau), v = (0, s, kappa),
K = R^n x K* x R_+, and
    Q(u) = (Px + A'y + tau q,  -Ax + tau b,  -(1/tau) x'Px - q'x - b'y).
Residual map (Sec. 2.3, eq. residual-map):  R(z) = Q(Pi z) - Pi z + z.
Normalised residual (eq. normalized-residual):  N(z) = R(z) / |z_N|.
Data derivative (Sec. 2.4, "with respect to the data"): D_theta N = D_theta Q(Pi z)/|z_N|
and its adjoint D_theta Q' [w] = (P~, A~, q~, b~).
Variable derivative (Sec. 2.4, "with respect to the variables"):
    F = D_z N = (1/z_N) (D_u Q(Pi z) DPi(z) - DPi(z) + I),
    D_u Q(u) = [[P, A', q], [-A, 0, b], [(-2/tau) x'P - q', -b', (1/tau^2) x'Px]].
Solution construction (Sec. 2.4, "Solution construction"):
    phi(z) = (z_x, Pi_{K*}(z_y), Pi_{K*}(z_y) - z_y) / z_N  and its Jacobian D phi.
"""
from __future__ import annotations

import numpy as np

from . import cones as C


class Embedding:
    """Operators at a fixed point z for a fixed instance (P, A, q, b, K)."""

    def __init__(self, qcp, z=None):
        self.qcp = qcp
        self.n, self.m = qcp.n, qcp.m
        self.N = self.n + self.m + 1
        if z is None:
            z = point_from_solution(qcp.x, qcp.y, qcp.s)
        self.z = np.asarray(z, dtype=np.float64)
        n, m = self.n, self.m
        zx, zy, zN = self.z[:n], self.z[n:n + m], self.z[-1]
        self.zN = zN
        # Pi z = (z_x, Pi_{K*}(z_y), max(z_N, 0))
        self.u = np.concatenate([zx, C.proj_dual(zy, qcp.cones), [max(zN, 0.0)]])
        self.J = C.DualJacobian(zy, qcp.cones)
        self.dtau = 1.0 if zN > 0 else 0.0
        ux, tau = self.u[:n], self.u[-1]
        self.Px = qcp.P @ ux
        self.xPx = float(ux @ self.Px)

    # ---- DPi(z) ---------------------------------------------------------------------
    def dpi(self, v):
        n, m = self.n, self.m
        return np.concatenate([v[:n], self.J.apply(v[n:n + m]), [self.dtau * v[-1]]])

    # ---- D_u Q(Pi z) and its transpose ----------------------------------------------
    def dq(self, w):
        q = self.qcp
        n, m = self.n, self.m
        ux, uy, tau = self.u[:n], self.u[n:n + m], self.u[-1]
        wx, wy, wN = w[:n], w[n:n + m], w[-1]
        top = q.P @ wx + q.A.T @ wy + q.q * wN
        mid = -(q.A @ wx) + q.b * wN
        bot = ((-2.0 / tau) * self.Px - q.q) @ wx - q.b @ wy + (self.xPx / tau ** 2) * wN
        return np.concatenate([top, mid, [bot]])

    def dq_t(self, r):
        q = self.qcp
        n, m = self.n, self.m
        tau = self.u[-1]
        rx, ry, rN = r[:n], r[n:n + m], r[-1]
        cvec = (-2.0 / tau) * self.Px - q.q
        top = q.P @ rx - q.A.T @ ry + cvec * rN
        mid = q.A @ rx - q.b * rN
        bot = q.q @ rx + q.b @ ry + (self.xPx / tau ** 2) * rN
        return np.concatenate([top, mid, [bot]])

    # ---- F = D_z N and F' -----------------------------------------------------------
    def F(self, v):
        w = self.dpi(v)
        return (self.dq(w) - w + v) / self.zN

    def FT(self, r):
        # DPi is symmetric: F' r = (DPi DQ' r - DPi r + r) / z_N
        return (self.dpi(self.dq_t(r)) - self.dpi(r) + r) / self.zN

    def F_dense(self):
        M = np.empty((self.N, self.N))
        for j in range(self.N):
            e = np.zeros(self.N)
            e[j] = 1.0
            M[:, j] = self.F(e)
        return M

    # ---- D_theta N and its adjoint ----------------------------------------------------
    def dtheta(self, dP, dA, dq, db):
        """D_theta N(z)[dtheta] with dP, dA given as values on the stored patterns."""
        q = self.qcp
        n, m = self.n, self.m
        x, y, tau = self.u[:n], self.u[n:n + m], self.u[-1]
        dPm = _with_values(q.P, dP)
        dAm = _with_values(q.A, dA)
        dPx = dPm @ x
        top = dPx + dAm.T @ y + tau * dq
        mid = -(dAm @ x) + tau * db
        bot = (-1.0 / tau) * (x @ dPx) - dq @ x - db @ y
        return np.concatenate([top, mid, [bot]]) / abs(self.zN)

    def dtheta_t(self, w):
        """D_theta N(z)' [w], returned on the stored patterns of P and A."""
        q = self.qcp
        n, m = self.n, self.m
        x, y, tau = self.u[:n], self.u[n:n + m], self.u[-1]
        wx, wy, wN = w[:n], w[n:n + m], w[-1]
        Pi, Pj = _coords(q.P)
        Ai, Aj = _coords(q.A)
        dP = 0.5 * (wx[Pi] * x[Pj] + x[Pi] * wx[Pj]) - (wN / tau) * x[Pi] * x[Pj]
        dA = y[Ai] * wx[Aj] - wy[Ai] * x[Aj]
        dq = tau * wx - wN * x
        db = tau * wy - wN * y
        s = 1.0 / abs(self.zN)
        return dP * s, dA * s, dq * s, db * s

    # ---- phi and D phi -----------------------------------------------------------------
    def dphi(self, dz):
        n, m = self.n, self.m
        x, y = self.u[:n], self.u[n:n + m]
        s = y - self.z[n:n + m]
        Jdy = self.J.apply(dz[n:n + m])
        dzN = dz[-1]
        return (dz[:n] - dzN * x, Jdy - dzN * y, Jdy - dz[n:n + m] - dzN * s)

    def dphi_t(self, gx, gy, gs):
        n, m = self.n, self.m
        x, y = self.u[:n], self.u[n:n + m]
        s = y - self.z[n:n + m]
        mid = self.J.apply(gy + gs) - gs
        return np.concatenate([gx, mid, [-(x @ gx) - (y @ gy) - (s @ gs)]])


def point_from_solution(x, y, s):
    """z = M^{-1}(u, v) = u - v with u = (x, y, 1), v = (0, s, 0) (Sec. 3.1)."""
    return np.concatenate([x, y - s, [1.0]])


def Q_map(qcp, u):
    n, m = qcp.n, qcp.m
    x, y, tau = u[:n], u[n:n + m], u[-1]
    Px = qcp.P @ x
    return np.concatenate([Px + qcp.A.T @ y + tau * qcp.q,
                           -(qcp.A @ x) + tau * qcp.b,
                           [-(1.0 / tau) * (x @ Px) - qcp.q @ x - qcp.b @ y]])


def proj_K(qcp, z):
    n, m = qcp.n, qcp.m
    return np.concatenate([z[:n], C.proj_dual(z[n:n + m], qcp.cones), [max(z[-1], 0.0)]])


def residual(qcp, z):
    """R(z) = Q(Pi z) - Pi z + z (eq. residual-map)."""
    u = proj_K(qcp, z)
    return Q_map(qcp, u) - u + z


def normalized_residual(qcp, z):
    return residual(qcp, z) / abs(z[-1])


def phi(qcp, z):
    n, m = qcp.n, qcp.m
    py = C.proj_dual(z[n:n + m], qcp.cones)
    return z[:n] / z[-1], py / z[-1], (py - z[n:n + m]) / z[-1]


def _coords(M):
    rows = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))
    return rows, M.indices.astype(np.int64)


def _with_values(M, vals):
    out = M.copy()
    out.data = np.asarray(vals, dtype=np.float64).copy()
    return out


def with_data(qcp, dP=None, dA=None, dq=None, db=None, h=1.0):
    """A copy of the instance with theta + h * dtheta (same patterns, same solution
    fields, which are then stale)."""
    import copy
    out = copy.copy(qcp)
    out.P = _with_values(qcp.P, qcp.P.data + (h * dP if dP is not None else 0.0))
    out.A = _with_values(qcp.A, qcp.A.data + (h * dA if dA is not None else 0.0))
    out.q = qcp.q + (h * dq if dq is not None else 0.0)
    out.b = qcp.b + (h * db if db is not None else 0.0)
    return out
