"""Projections onto the dual cones K* and their Jacobians, written from Appendix A
("Cones, projections, and derivatives").

The embedding projects the y-part of z onto the DUAL cone K* (Sec. 2.1: K = R^n x K* x R_+),
so per block:
  zero cone        -> dual is R: projection = identity, Jacobian = I   (App. A, "Zero cone")
  nonnegative cone -> self-dual                                        (App. A, "Nonnegative cone")
  second-order     -> self-dual                                        (App. A, "Second-order cone")
  PSD (svec)       -> self-dual                                        (App. A, "Positive semidefinite cone")
  exponential      -> dual exponential cone via Moreau:
                      Pi_{exp*}(z) = z + Pi_exp(-z), DPi_{exp*}(z) = I - DPi_exp(-z)
                                                                       (App. A, "Dual exponential cone")
  power (K_pow,a)  -> dual power cone via Moreau, as for the exponential cone
                                                                       (App. A, "Dual power cone")
  dual power       -> its dual is K_pow,a itself                       (App. A, "Power cone")
Readings where the appendix is silent or garbled:
  * at kinks the cases are tested in the listed order with closed inequalities
    (nonneg: 1{z > 0}; SOC: ||u|| <= -t -> 0, ||u|| <= t -> I, else the formula);
  * PSD blocks are stored as svec (lower triangle, column-major, off-diagonals x sqrt 2) so the
    projection is Euclidean in R^{k(k+1)/2} and the Jacobian is symmetric;
  * PSD: with no negative eigenvalue B is all ones, with all negative it is all zeros;
  * exponential 4x4 matrix, entry (2,2): 1 + mu x^2 e^{x/y} / y^3 (the Hessian of y e^{x/y},
    the printed "1 + -" is read as "+");
  * the exponential projection objective is the squared distance.
"""
from __future__ import annotations

import math

import numpy as np

SQRT2 = math.sqrt(2.0)


# ----------------------------------------------------------------------------------------
# nonnegative cone (App. A, "Nonnegative cone")
# ----------------------------------------------------------------------------------------

def proj_nonneg(z):
    return np.where(z >= 0, z, 0.0)


def jac_nonneg_diag(z):
    return np.where(z > 0, 1.0, 0.0)


# ----------------------------------------------------------------------------------------
# second-order cone {(t, u): ||u|| <= t} (App. A, "Second-order cone")
# ----------------------------------------------------------------------------------------

def proj_soc(z):
    t, u = z[0], z[1:]
    nu = np.linalg.norm(u)
    if nu <= -t:
        return np.zeros_like(z)
    if nu <= t:
        return z.copy()
    c = 0.5 * (1.0 + t / nu)
    return c * np.concatenate([[nu], u])


def jac_soc(z):
    """Dense k x k Jacobian. Third case: (dt, du) -> 1/(2||u||) [||u|| dt + u'du ;
    u dt + (t + ||u||) du - (t/||u||^2)(u'du) u]."""
    k = z.size
    t, u = z[0], z[1:]
    nu = np.linalg.norm(u)
    if nu <= -t:
        return np.zeros((k, k))
    if nu <= t:
        return np.eye(k)
    J = np.zeros((k, k))
    J[0, 0] = nu
    J[0, 1:] = u
    J[1:, 0] = u
    J[1:, 1:] = (t + nu) * np.eye(k - 1) - (t / nu ** 2) * np.outer(u, u)
    return J / (2.0 * nu)


# ----------------------------------------------------------------------------------------
# PSD cone on svec coordinates (App. A, "Positive semidefinite cone")
# ----------------------------------------------------------------------------------------

def svec(Z):
    k = Z.shape[0]
    out = np.empty(k * (k + 1) // 2)
    t = 0
    for j in range(k):
        for i in range(j, k):
            out[t] = Z[i, j] if i == j else SQRT2 * Z[i, j]
            t += 1
    return out


def smat(v, k):
    Z = np.empty((k, k))
    t = 0
    for j in range(k):
        for i in range(j, k):
            if i == j:
                Z[i, i] = v[t]
            else:
                Z[i, j] = Z[j, i] = v[t] / SQRT2
            t += 1
    return Z


def psd_order(rows):
    k = int(round((math.sqrt(8 * rows + 1) - 1) / 2))
    assert k * (k + 1) // 2 == rows
    return k


def eig_desc(Z):
    """Eigen-decomposition with eigenvalues in descending order, as the appendix orders
    them (library routine: numpy.linalg.eigh)."""
    lam, V = np.linalg.eigh(Z)
    return lam[::-1].copy(), V[:, ::-1].copy()


def proj_psd(v):
    """Pi(Z) = sum_i max(0, lambda_i) v_i v_i'."""
    k = psd_order(v.size)
    lam, V = eig_desc(smat(v, k))
    return svec((V * np.maximum(lam, 0.0)) @ V.T)


def psd_B(lam):
    """B from the appendix with k = min{k : lambda_k < 0} on descending eigenvalues
    (0-based here: indices < kk are the nonnegative group)."""
    n = lam.size
    neg = np.nonzero(lam < 0)[0]
    kk = int(neg[0]) if neg.size else n
    B = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i < kk and j < kk:
                B[i, j] = 1.0
            elif i >= kk and j >= kk:
                B[i, j] = 0.0
            elif i < kk <= j:
                B[i, j] = lam[i] / (lam[i] - lam[j])
            else:
                B[i, j] = lam[j] / (lam[j] - lam[i])
    return B


def psd_factors(v):
    k = psd_order(v.size)
    lam, V = eig_desc(smat(v, k))
    return V, psd_B(lam), lam


def jac_psd_apply(V, B, dv):
    """DPi(Z)[dZ] = V (B o (V' dZ V)) V' in svec coordinates."""
    k = V.shape[0]
    dZ = smat(dv, k)
    return svec(V @ (B * (V.T @ dZ @ V)) @ V.T)


def jac_psd(v):
    V, B, _ = psd_factors(v)
    r = v.size
    J = np.empty((r, r))
    for c in range(r):
        e = np.zeros(r)
        e[c] = 1.0
        J[:, c] = jac_psd_apply(V, B, e)
    return J


# ----------------------------------------------------------------------------------------
# exponential cone (App. A, "Exponential cone")
#   K_exp  = {(x,y,z): y e^{x/y} <= z, y > 0} U {(x,0,z): x <= 0, z >= 0}
#   K_exp* = {(u,v,w): u < 0, -u e^{v/u} <= e w} U {(0,v,w): v >= 0, w >= 0}
#   polar  = -K_exp*
# ----------------------------------------------------------------------------------------

def _safe_exp(a):
    return math.exp(a) if a < 700.0 else math.inf


def in_exp(p):
    x, y, z = p
    if y > 0:
        return y * _safe_exp(x / y) <= z
    return y == 0 and x <= 0 and z >= 0


def in_exp_dual(p):
    u, v, w = p
    if u < 0:
        return -u * _safe_exp(v / u) <= math.e * w
    return u == 0 and v >= 0 and w >= 0


def in_exp_polar(p):
    return in_exp_dual(-np.asarray(p))


def _ray_dir(r):
    """d1(r) = (r, 1, e^r) scaled to avoid overflow: the boundary ray of K_exp with
    x/y = r, y > 0."""
    sc = max(1.0, abs(r), math.exp(min(r, 700.0)))
    return np.array([r / sc, 1.0 / sc, math.exp(min(r, 700.0)) / sc])


def _exp_case4(p):
    """Projection onto the smooth boundary part (the minimisation problem of
    eq. exp-system): hat p = yhat (r, 1, e^r). For a fixed r the best yhat is
    <p, d1>/||d1||^2, so r maximises g(r) = <p, d1(r)>/||d1(r)||. A grid scan finds the
    maximiser's neighbourhood; bisection on g'(r) then pins r to full precision."""
    p = np.asarray(p, dtype=np.float64)

    def g(r):
        er = np.exp(np.minimum(r, 700.0))
        sc = np.maximum(np.maximum(1.0, np.abs(r)), er)
        d0, d1_, d2_ = r / sc, 1.0 / sc, er / sc
        return (p[0] * d0 + p[1] * d1_ + p[2] * d2_) / np.sqrt(d0 * d0 + d1_ * d1_ + d2_ * d2_)

    def dg(r):
        # sign of d/dr <p,d>/||d|| with d = (r,1,e^r) and d' = (1,0,e^r), up to a
        # positive factor: <p,d'>||d||^2 - <p,d><d,d'>
        er = math.exp(min(r, 700.0))
        sc = max(1.0, abs(r), er)
        d = np.array([r, 1.0, er]) / sc
        dd = np.array([1.0, 0.0, er]) / sc
        return float(p @ dd) * float(d @ d) - float(p @ d) * float(d @ dd)

    lo, hi, step = -40.0, 40.0, 0.01
    while True:
        grid = np.arange(lo, hi + step / 2, step)
        vals = g(grid)
        kmax = int(np.argmax(vals))
        if 0 < kmax < grid.size - 1:
            break
        if kmax == 0:
            lo -= 80.0
        else:
            if hi >= 690.0:
                break
            hi = min(hi + 80.0, 690.0)
    a = float(grid[max(kmax - 1, 0)])
    b = float(grid[min(kmax + 1, grid.size - 1)])
    fa, fb = dg(a), dg(b)
    if fa * fb > 0:
        r = float(grid[kmax])
    else:
        for _ in range(200):
            mid = 0.5 * (a + b)
            if mid <= a or mid >= b:
                break
            fm = dg(mid)
            if fm == 0:
                a = b = mid
                break
            if (fm > 0) == (fa > 0):
                a, fa = mid, fm
            else:
                b = mid
        r = 0.5 * (a + b)
    er = math.exp(r)
    d1 = np.array([r, 1.0, er])
    yhat = float(p @ d1) / float(d1 @ d1)
    phat = yhat * d1
    d2 = np.array([er, (1.0 - r) * er, -1.0])
    mu = float(p @ d2) / float(d2 @ d2)
    return phat, r, yhat, mu


def proj_exp(p):
    """Pi_exp by the appendix's four cases, tested in the listed order."""
    p = np.asarray(p, dtype=np.float64)
    x, y, z = p
    if in_exp(p):
        return p.copy()
    if in_exp_polar(p):
        return np.zeros(3)
    if x < 0 and y < 0:
        return np.array([x, 0.0, max(z, 0.0)])
    return _exp_case4(p)[0]


def jac_exp(p):
    """DPi_exp(p) (App. A, exponential cone derivative cases)."""
    p = np.asarray(p, dtype=np.float64)
    x, y, z = p
    if in_exp(p):
        return np.eye(3)
    if in_exp_polar(p):
        return np.zeros((3, 3))
    if x < 0 and y < 0:
        return np.diag([1.0, 0.0, 1.0 if z > 0 else 0.0])
    phat, r, yhat, mu = _exp_case4(p)
    xs, ys = phat[0], phat[1]
    e = math.exp(xs / ys)
    J4 = np.array([
        [1 + mu * e / ys, -mu * xs * e / ys ** 2, 0.0, e],
        [-mu * xs * e / ys ** 2, 1 + mu * xs ** 2 * e / ys ** 3, 0.0, (1 - xs / ys) * e],
        [0.0, 0.0, 1.0, -1.0],
        [e, (1 - xs / ys) * e, -1.0, 0.0],
    ])
    return np.linalg.inv(J4)[:3, :3]


def proj_exp_dual(z):
    return np.asarray(z) + proj_exp(-np.asarray(z))


def jac_exp_dual(z):
    return np.eye(3) - jac_exp(-np.asarray(z))


# ----------------------------------------------------------------------------------------
# power cone (App. A, "Power cone"), 0 < a < 1
#   K_pow,a  = {(x,y,z): x^a y^(1-a) >= |z|, x >= 0, y >= 0}
#   K_pow,a* = {(u,v,w): (u/a)^a (v/(1-a))^(1-a) >= |w|, u >= 0, v >= 0}
#   polar    = -K_pow,a*
# ----------------------------------------------------------------------------------------

def in_pow(p, a):
    x, y, z = p
    return x >= 0 and y >= 0 and x ** a * y ** (1.0 - a) >= abs(z)


def in_pow_dual(p, a):
    u, v, w = p
    return u >= 0 and v >= 0 and (u / a) ** a * (v / (1.0 - a)) ** (1.0 - a) >= abs(w)


def in_pow_polar(p, a):
    return in_pow_dual(-np.asarray(p, dtype=np.float64), a)


def _half_root(x, t):
    """(x + sqrt(x^2 + t)) / 2 for t >= 0; for x < 0 as t / (2 (sqrt(x^2 + t) - x)), the same
    number without the cancellation."""
    s = math.sqrt(x * x + t)
    return 0.5 * (x + s) if x >= 0 else 0.5 * t / (s - x)


def _pow_f(x, y, z, a, r):
    """f_x(r), f_y(r) of eq. pow-system."""
    az = abs(z)
    fx = _half_root(x, 4.0 * a * r * (az - r))
    fy = _half_root(y, 4.0 * (1.0 - a) * r * (az - r))
    return fx, fy


def _pow_root(p, a):
    """The solution r in (0, |z|) of r = f_x(r)^a f_y(r)^(1-a) (eq. pow-system). Outside
    K and its polar, h(r) = f_x^a f_y^(1-a) - r is positive just above 0 and negative at
    |z|; plain bisection on the sign of h until the bracket stops shrinking."""
    x, y, z = (float(t) for t in p)
    lo, hi = 0.0, abs(z)

    def h(r):
        fx, fy = _pow_f(x, y, z, a, r)
        return fx ** a * fy ** (1.0 - a) - r

    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if h(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def proj_pow(p, a):
    """Pi_pow,a by the appendix's four cases, tested in the listed order."""
    p = np.asarray(p, dtype=np.float64)
    x, y, z = p
    if in_pow(p, a):
        return p.copy()
    if in_pow_polar(p, a):
        return np.zeros(3)
    if z == 0.0:
        return np.array([max(x, 0.0), max(y, 0.0), 0.0])
    r = _pow_root(p, a)
    fx, fy = _pow_f(x, y, z, a, r)
    return np.array([fx, fy, math.copysign(r, z)])


def jac_pow(p, a):
    """DPi_pow,a(p) (App. A, power cone derivative cases; the z != 0 case is the closed form
    the appendix takes from Hien's Theorem 3.1)."""
    p = np.asarray(p, dtype=np.float64)
    x, y, z = p
    if in_pow(p, a):
        return np.eye(3)
    if in_pow_polar(p, a):
        return np.zeros((3, 3))
    if z == 0.0:
        if x > 0 and y < 0:
            d = 1.0 if a > 0.5 else (0.0 if a < 0.5 else x / (2.0 * abs(y) + x))
        elif x < 0 and y > 0:
            d = 1.0 if a < 0.5 else (0.0 if a > 0.5 else y / (2.0 * abs(x) + y))
        else:
            d = 0.0
        return np.diag([1.0 if x > 0 else 0.0, 1.0 if y > 0 else 0.0, d])
    r = _pow_root(p, a)
    fx, fy = _pow_f(x, y, z, a, r)
    az, sz = abs(z), math.copysign(1.0, z)
    gx, gy = 2.0 * fx - x, 2.0 * fy - y
    T = -(a * x / gx + (1.0 - a) * y / gy)
    L = 2.0 * (az - r) / (az + (az - 2.0 * r) * (a * x / gx + (1.0 - a) * y / gy))
    J = np.empty((3, 3))
    J[0, 0] = 0.5 + x / (2.0 * gx) + a * a * (az - 2.0 * r) * r * L / gx ** 2
    J[0, 1] = J[1, 0] = (a - a * a) * (az - 2.0 * r) * r * L / (gx * gy)
    J[0, 2] = J[2, 0] = sz * a * r * L / gx
    J[1, 1] = 0.5 + y / (2.0 * gy) + (1.0 - a) ** 2 * (az - 2.0 * r) * r * L / gy ** 2
    J[1, 2] = J[2, 1] = sz * (1.0 - a) * r * L / gy
    J[2, 2] = r / az + (r / az) * T * L
    return J


def proj_pow_dual(zv, a):
    """Pi onto K_pow,a* by Moreau (App. A, "Dual power cone"): z + Pi_pow,a(-z)."""
    return np.asarray(zv, dtype=np.float64) + proj_pow(-np.asarray(zv, dtype=np.float64), a)


def jac_pow_dual(zv, a):
    return np.eye(3) - jac_pow(-np.asarray(zv, dtype=np.float64), a)


# ----------------------------------------------------------------------------------------
# product cone K* in this project's row order: zero, nonneg, SOC..., PSD..., exp...,
# power..., dual power... For a power cone K_pow,a the dual cone K* is K_pow,a* (projected by
# Moreau); for a dual power cone K_pow,a* it is K_pow,a itself.
# ----------------------------------------------------------------------------------------

def blocks(cones):
    """Yield (kind, start, size) for each block of rows."""
    off = 0
    if cones.n_zero:
        yield ("zero", off, cones.n_zero)
        off += cones.n_zero
    if cones.n_nonneg:
        yield ("nonneg", off, cones.n_nonneg)
        off += cones.n_nonneg
    for k in cones.soc:
        yield ("soc", off, k)
        off += k
    for k in cones.psd:
        r = k * (k + 1) // 2
        yield ("psd", off, r)
        off += r
    for _ in range(cones.n_exp):
        yield ("exp", off, 3)
        off += 3
    for a in getattr(cones, "pow", ()):
        yield (("pow", a), off, 3)
        off += 3
    for a in getattr(cones, "dpow", ()):
        yield (("dpow", a), off, 3)
        off += 3


def proj_dual(zy, cones):
    """Pi_{K*}(z_y)."""
    out = np.empty_like(zy)
    for kind, a, r in blocks(cones):
        seg = zy[a:a + r]
        if kind == "zero":
            out[a:a + r] = seg
        elif kind == "nonneg":
            out[a:a + r] = proj_nonneg(seg)
        elif kind == "soc":
            out[a:a + r] = proj_soc(seg)
        elif kind == "psd":
            out[a:a + r] = proj_psd(seg)
        elif kind == "exp":
            out[a:a + r] = proj_exp_dual(seg)
        elif kind[0] == "pow":        # K* = K_pow,a*
            out[a:a + r] = proj_pow_dual(seg, kind[1])
        else:                         # dual power cone: K* = K_pow,a
            out[a:a + r] = proj_pow(seg, kind[1])
    return out


class DualJacobian:
    """J = DPi_{K*}(z_y), block diagonal. Blocks of one kind and size are stacked so that
    applying J is a handful of batched products."""

    def __init__(self, zy, cones):
        self.m = zy.size
        diag_rows, diag_vals = [], []
        dense = {}   # size -> (starts, mats)
        psd = {}     # k -> (starts, V, B)
        for kind, a, r in blocks(cones):
            seg = zy[a:a + r]
            if kind == "zero":
                diag_rows.append(np.arange(a, a + r))
                diag_vals.append(np.ones(r))
            elif kind == "nonneg":
                diag_rows.append(np.arange(a, a + r))
                diag_vals.append(jac_nonneg_diag(seg))
            elif kind == "soc":
                dense.setdefault(r, ([], []))
                dense[r][0].append(a)
                dense[r][1].append(jac_soc(seg))
            elif kind == "exp" or kind[0] in ("pow", "dpow"):
                dense.setdefault(3, ([], []))
                dense[3][0].append(a)
                if kind == "exp":
                    dense[3][1].append(jac_exp_dual(seg))
                elif kind[0] == "pow":
                    dense[3][1].append(jac_pow_dual(seg, kind[1]))
                else:
                    dense[3][1].append(jac_pow(seg, kind[1]))
            else:
                k = psd_order(r)
                V, B, _ = psd_factors(seg)
                psd.setdefault(k, ([], [], []))
                psd[k][0].append(a)
                psd[k][1].append(V)
                psd[k][2].append(B)
        self.diag_rows = np.concatenate(diag_rows) if diag_rows else np.zeros(0, int)
        self.diag_vals = np.concatenate(diag_vals) if diag_vals else np.zeros(0)
        self.dense = {r: (np.asarray(s), np.stack(M)) for r, (s, M) in dense.items()}
        self.psd = {}
        for k, (s, V, B) in psd.items():
            r = k * (k + 1) // 2
            # svec <-> smat index maps for batched unpack/pack
            I, Jc, W = [], [], []
            for j in range(k):
                for i in range(j, k):
                    I.append(i)
                    Jc.append(j)
                    W.append(1.0 if i == j else SQRT2)
            self.psd[k] = (np.asarray(s), np.stack(V), np.stack(B),
                           (np.asarray(I), np.asarray(Jc), np.asarray(W), r))

    def apply(self, v):
        out = np.zeros_like(v)
        out[self.diag_rows] = self.diag_vals * v[self.diag_rows]
        for r, (starts, M) in self.dense.items():
            idx = starts[:, None] + np.arange(r)[None, :]
            out[idx] = np.einsum("bij,bj->bi", M, v[idx])
        for k, (starts, V, B, (I, Jc, W, r)) in self.psd.items():
            idx = starts[:, None] + np.arange(r)[None, :]
            vals = v[idx]
            Z = np.zeros((starts.size, k, k))
            Z[:, I, Jc] = vals / W
            Z[:, Jc, I] = vals / W
            T = np.transpose(V, (0, 2, 1)) @ Z @ V
            Y = V @ (B * T) @ np.transpose(V, (0, 2, 1))
            out[idx] = Y[:, I, Jc] * W
        return out

    def dense_matrix(self):
        """Dense m x m J (small problems only)."""
        J = np.zeros((self.m, self.m))
        for c in range(self.m):
            e = np.zeros(self.m)
            e[c] = 1.0
            J[:, c] = self.apply(e)
        return J

    def diagonal(self):
        """diag(J). For a PSD block and the svec basis element of entry (i, j):
        <E, V(B o V'EV)V'> = sum_ab B_ab (V'EV)_ab^2, written out per entry."""
        d = np.zeros(self.m)
        d[self.diag_rows] = self.diag_vals
        for r, (starts, M) in self.dense.items():
            for a, Mb in zip(starts, M):
                d[a:a + r] = np.diag(Mb)
        for k, (starts, V, B, (I, Jc, W, r)) in self.psd.items():
            for bi, a in enumerate(starts):
                Vb, Bb = V[bi], B[bi]
                S = Vb * Vb
                D1 = S @ Bb @ S.T                      # (V_i^2)' B (V_j^2)
                U = Vb[I] * Vb[Jc]                     # rows: V_i o V_j
                D2 = np.einsum("ta,ab,tb->t", U, Bb, U)
                off = I != Jc
                d[a:a + r] = np.where(off, D1[I, Jc] + D2, D1[I, I])
        return d
