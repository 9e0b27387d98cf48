"""Seeded synthetic quadratic cone programs built around a known primal-dual solution.

This module only *draws* problem instances; it holds none of the derivative method's
arithmetic (no cone projections, no cone Jacobians, no embedding operator, no solver).
Both the CPU oracle and the GPU library consume the instances it produces.

Problem form (Sec. 2.1, eq. conic-pair):
    minimize  1/2 x'Px + q'x   s.t.  Ax + s = b,  s in K
    dual:     Px + A'y = -q,  y in K*
A complementary pair (s, y) is drawn per cone block, then q = -Px - A'y and b = Ax + s make
(x, y, s) satisfy the KKT conditions (Sec. 2.1, eq. kkt-conds) exactly up to rounding.

Row order of the cone (a layout convention of this project): zero, nonnegative, second-order
cones, PSD cones (svec: lower triangle, column-major, off-diagonal entries scaled by sqrt 2),
exponential cones, power cones, dual power cones (3 rows each, ordered (x, y, z) as in
Appendix A).

Seeds: numpy.random.default_rng([config_id, problem_idx, attempt]).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

SQRT2 = math.sqrt(2.0)


@dataclasses.dataclass
class Cones:
    n_zero: int = 0
    n_nonneg: int = 0
    soc: List[int] = dataclasses.field(default_factory=list)   # dimension of each SOC
    psd: List[int] = dataclasses.field(default_factory=list)   # order k of each PSD block
    n_exp: int = 0
    pow: List[float] = dataclasses.field(default_factory=list)   # alpha of each power cone
    dpow: List[float] = dataclasses.field(default_factory=list)  # alpha of each dual power cone

    @property
    def m(self) -> int:
        return (self.n_zero + self.n_nonneg + sum(self.soc)
                + sum(k * (k + 1) // 2 for k in self.psd) + 3 * self.n_exp
                + 3 * len(self.pow) + 3 * len(self.dpow))


@dataclasses.dataclass
class QCP:
    name: str
    n: int
    m: int
    P: sp.csr_matrix          # full symmetric pattern, sorted indices, int32 index arrays
    A: sp.csr_matrix          # m x n
    q: np.ndarray
    b: np.ndarray
    cones: Cones
    x: np.ndarray
    y: np.ndarray
    s: np.ndarray
    # a data perturbation on the stored patterns (dP symmetric on the pattern)
    dP: np.ndarray
    dA: np.ndarray
    dq: np.ndarray
    db: np.ndarray
    # a cotangent on (x, y, s)
    gx: np.ndarray
    gy: np.ndarray
    gs: np.ndarray
    tol: float = 1e-8
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n + self.m + 1


# ----------------------------------------------------------------------------------------
# small helpers (data layout only)
# ----------------------------------------------------------------------------------------

def svec(Z: np.ndarray) -> np.ndarray:
    """Lower triangle, column-major, off-diagonals times sqrt(2)."""
    k = Z.shape[0]
    out = []
    for j in range(k):
        for i in range(j, k):
            out.append(Z[i, j] if i == j else SQRT2 * Z[i, j])
    return np.asarray(out, dtype=np.float64)


def smat(v: np.ndarray, k: int) -> np.ndarray:
    Z = np.zeros((k, k))
    t = 0
    for j in range(k):
        for i in range(j, k):
            if i == j:
                Z[i, i] = v[t]
            else:
                Z[i, j] = Z[j, i] = v[t] / SQRT2
            t += 1
    return Z


def _csr(M) -> sp.csr_matrix:
    M = sp.csr_matrix(M)
    M.sum_duplicates()
    M.sort_indices()
    M.indptr = M.indptr.astype(np.int32)
    M.indices = M.indices.astype(np.int32)
    M.data = M.data.astype(np.float64)
    return M


def transpose_slots(M: sp.csr_matrix) -> np.ndarray:
    """For a structurally symmetric CSR matrix, slot t[k] holds entry (j, i) when slot k
    holds (i, j)."""
    n = M.shape[0]
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(M.indptr))
    cols = M.indices.astype(np.int64)
    key = rows * n + cols
    if key.size and bool(np.all(key[1:] > key[:-1])):  # canonical CSR: keys ascending
        if key.size == n * n:  # every entry stored: slot of (i, j) is i n + j
            return cols * n + rows
        return np.searchsorted(key, cols * n + rows)
    tkey = cols * n + rows
    order = np.argsort(key)
    pos = np.searchsorted(key[order], tkey)
    return order[pos]


def sparse_gaussian(rng, m, n, density, min_row_nnz=3) -> sp.csr_matrix:
    """Bernoulli(density) pattern with N(0,1) values. Rows with fewer than min_row_nnz
    entries are topped up and empty columns receive one entry: at the sparse densities of
    the larger workloads (about 5 entries per row) single-entry rows collide often enough
    to make the active constraints linearly dependent, i.e. the derivative undefined."""
    nnz = int(round(density * m * n))
    if nnz > 0:
        flat = rng.choice(m * n, size=nnz, replace=False) if m * n < 5e7 else \
            np.unique(rng.integers(0, m * n, size=int(nnz * 1.02) + 16))[:nnz]
        r = (flat // n).astype(np.int64)
        c = (flat % n).astype(np.int64)
    else:
        r = np.zeros(0, np.int64)
        c = np.zeros(0, np.int64)
    need = min(min_row_nnz, n)
    if m > 0 and need > 0:
        rowcnt = np.bincount(r, minlength=m)
        short = np.nonzero(rowcnt < need)[0]
        add_r, add_c = [], []
        used = set(zip(r[np.isin(r, short)].tolist(), c[np.isin(r, short)].tolist()))
        for i in short.tolist():
            have = {cc for (rr, cc) in used if rr == i}
            while len(have) < need:
                j = int(rng.integers(0, n))
                if j not in have:
                    have.add(j)
                    add_r.append(i)
                    add_c.append(j)
        r = np.concatenate([r, np.asarray(add_r, np.int64)])
        c = np.concatenate([c, np.asarray(add_c, np.int64)])
    colcnt = np.bincount(c, minlength=n)
    ec = np.nonzero(colcnt == 0)[0]
    if m > 0:
        r = np.concatenate([r, rng.integers(0, m, size=ec.size)])
        c = np.concatenate([c, ec])
    v = rng.standard_normal(r.size)
    M = sp.coo_matrix((v, (r, c)), shape=(m, n))
    return _csr(M)


def psd_from_factor(B: sp.spmatrix | np.ndarray, eps: float) -> sp.csr_matrix:
    if sp.issparse(B):
        P = (B @ B.T).tocsr()
    else:
        P = sp.csr_matrix(B @ B.T)
    if eps:
        P = P + eps * sp.identity(P.shape[0], format="csr")
    P = _csr(P)
    P = _csr((P + P.T) * 0.5)  # exact symmetry
    return P


def symmetric_on_pattern(rng, P: sp.csr_matrix, std: float) -> np.ndarray:
    g = std * rng.standard_normal(P.nnz)
    t = transpose_slots(P)
    return 0.5 * (g + g[t])


def random_orthogonal(rng, k) -> np.ndarray:
    G = rng.standard_normal((k, k))
    Qm, R = np.linalg.qr(G)
    return Qm * np.sign(np.diag(R))


# ----------------------------------------------------------------------------------------
# complementary (s, y) pairs per cone block
# ----------------------------------------------------------------------------------------

def _soc_pair(rng, k, state):
    """state: 's_int' (s interior, y = 0), 'y_int' (s = 0, y interior), 'bnd' (both on
    the boundary, orthogonal). Returns s, y, hard codimension."""
    if k == 1:
        if state == 's_int':
            return np.array([rng.uniform(0.1, 1)]), np.zeros(1), 0
        return np.zeros(1), np.array([rng.uniform(0.1, 1)]), 1
    u = rng.standard_normal(k - 1)
    nu = np.linalg.norm(u)
    if state == 's_int':
        s = np.concatenate([[nu + rng.uniform(0.1, 1)], u])
        return s, np.zeros(k), 0
    if state == 'y_int':
        y = np.concatenate([[nu + rng.uniform(0.1, 1)], u])
        return np.zeros(k), y, k
    sig, alp = rng.uniform(0.1, 1, size=2)
    s = sig * np.concatenate([[nu], u])
    y = alp * np.concatenate([[nu], -u])
    return s, y, 1


def _psd_pair(rng, k, j):
    """rank(Y) = j, rank(S) = k - j, sharing eigenvectors (complementary)."""
    U = random_orthogonal(rng, k)
    om = rng.uniform(0.1, 1, size=j)
    sg = rng.uniform(0.1, 1, size=k - j)
    Y = (U[:, :j] * om) @ U[:, :j].T
    S = (U[:, j:] * sg) @ U[:, j:].T
    return svec(S), svec(Y), j * (j + 1) // 2


def _exp_pair(rng, state):
    """Complementary pair for the exponential cone: s in K_exp, y in K_exp*, s'y = 0."""
    if state == 's_int':
        r = rng.uniform(-2, 2)
        yy = rng.uniform(0.1, 1)
        s = np.array([yy * r, yy, yy * math.exp(r) + rng.uniform(0.1, 1)])
        return s, np.zeros(3), 0, {}
    if state == 'y_int':
        u = -rng.uniform(0.1, 1)
        v = rng.uniform(-1, 1)
        w = -u * math.exp(v / u - 1.0) + rng.uniform(0.1, 1)
        return np.zeros(3), np.array([u, v, w]), 3, {}
    r = rng.uniform(-2, 2)
    s2, mu = rng.uniform(0.1, 1, size=2)
    er = math.exp(r)
    s = s2 * np.array([r, 1.0, er])
    y = mu * np.array([-er, (r - 1.0) * er, 1.0])
    return s, y, 1, {"r": r, "s2": s2, "mu": mu}


def _pow_surface_pair(rng, a):
    """A boundary point w = (x, y, +-x^a y^(1-a)) of K_pow,a and the normal
    n = (a|z|/x, (1-a)|z|/y, -sign z) there, which lies on the boundary of K_pow,a* and is
    orthogonal to w (x^a y^(1-a) is homogeneous of degree one)."""
    x, y = rng.uniform(0.3, 2.0, size=2)
    zz = x ** a * y ** (1.0 - a) * (1.0 if rng.uniform() < 0.5 else -1.0)
    nrm = np.array([a * abs(zz) / x, (1.0 - a) * abs(zz) / y, -math.copysign(1.0, zz)])
    return np.array([x, y, zz]), nrm


def _pow_pair(rng, a, state, dual):
    """Complementary pair for a power cone (dual=False: s in K_pow,a, y in K_pow,a*) or a
    dual power cone (dual=True: s in K_pow,a*, y in K_pow,a). Returns s, y, hard codim."""
    if state == 's_int' or state == 'y_int':
        u, v = rng.uniform(0.3, 2.0, size=2)
        interior_of_k = (state == 's_int') != dual   # the vector drawn lies in int K_pow,a
        lim = u ** a * v ** (1.0 - a) if interior_of_k else \
            (u / a) ** a * (v / (1.0 - a)) ** (1.0 - a)
        w = rng.uniform(-0.8, 0.8) * lim
        vec = np.array([u, v, w])
        if state == 's_int':
            return vec, np.zeros(3), 0
        return np.zeros(3), vec, 3
    pt, nrm = _pow_surface_pair(rng, a)
    mu = rng.uniform(0.1, 1.0)
    if not dual:
        return pt, mu * nrm, 1
    return mu * nrm, pt, 1


# ----------------------------------------------------------------------------------------
# generic builder
# ----------------------------------------------------------------------------------------

def build(rng, name, n, cones: Cones, *, A_density, P, nonneg_active=None, soc_states=None,
          psd_ranks=None, exp_states=None, pow_states=None, pert_std=1e-2, tol=1e-8,
          A=None) -> QCP:
    m = cones.m
    if A is None:
        A = sparse_gaussian(rng, m, n, A_density)
    x = rng.standard_normal(n)
    s_parts, y_parts = [], []
    codim = 0
    # zero cone rows: s = 0, y free
    s_parts.append(np.zeros(cones.n_zero))
    y_parts.append(rng.standard_normal(cones.n_zero))
    codim += cones.n_zero
    # nonnegative rows
    nn = cones.n_nonneg
    if nonneg_active is None:
        nonneg_active = nn // 2
    nonneg_active = int(min(max(nonneg_active, 0), nn))
    act = np.zeros(nn, dtype=bool)
    act[rng.permutation(nn)[:nonneg_active]] = True
    s_nn = np.where(act, 0.0, rng.uniform(0.1, 1, size=nn))
    y_nn = np.where(act, rng.uniform(0.1, 1, size=nn), 0.0)
    s_parts.append(s_nn)
    y_parts.append(y_nn)
    codim += nonneg_active
    meta = {"nonneg_active": nonneg_active, "soc_states": [], "psd_ranks": [],
            "exp_states": [], "exp_params": []}
    for i, k in enumerate(cones.soc):
        st = soc_states[i] if soc_states is not None else ('s_int', 'y_int', 'bnd')[i % 3]
        s_, y_, c_ = _soc_pair(rng, k, st)
        s_parts.append(s_)
        y_parts.append(y_)
        codim += c_
        meta["soc_states"].append(st)
    for i, k in enumerate(cones.psd):
        j = psd_ranks[i] if psd_ranks is not None else k // 2
        s_, y_, c_ = _psd_pair(rng, k, j)
        s_parts.append(s_)
        y_parts.append(y_)
        codim += c_
        meta["psd_ranks"].append(j)
    for i in range(cones.n_exp):
        st = exp_states[i] if exp_states is not None else ('s_int', 'y_int', 'bnd')[i % 3]
        s_, y_, c_, prm = _exp_pair(rng, st)
        s_parts.append(s_)
        y_parts.append(y_)
        codim += c_
        meta["exp_states"].append(st)
        meta["exp_params"].append(prm)
    npow = len(cones.pow) + len(cones.dpow)
    for i, (a_, dual) in enumerate([(a_, False) for a_ in cones.pow] +
                                   [(a_, True) for a_ in cones.dpow]):
        st = pow_states[i] if pow_states is not None else ('s_int', 'y_int', 'bnd')[i % 3]
        s_, y_, c_ = _pow_pair(rng, a_, st, dual)
        s_parts.append(s_)
        y_parts.append(y_)
        codim += c_
        meta.setdefault("pow_states", []).append(st)
    del npow
    s = np.concatenate(s_parts) if s_parts else np.zeros(0)
    y = np.concatenate(y_parts) if y_parts else np.zeros(0)
    assert s.size == m and y.size == m
    q = -(P @ x) - A.T @ y
    b = A @ x + s
    dP = symmetric_on_pattern(rng, P, pert_std)
    dA = pert_std * rng.standard_normal(A.nnz)
    dq = pert_std * rng.standard_normal(n)
    db = pert_std * rng.standard_normal(m)
    gx = rng.standard_normal(n)
    gy = np.zeros(m)
    gs = np.zeros(m)
    meta["face_codim"] = codim
    return QCP(name=name, n=n, m=m, P=P, A=A, q=np.asarray(q, dtype=np.float64),
               b=np.asarray(b, dtype=np.float64), cones=cones, x=x, y=y, s=s,
               dP=dP, dA=dA, dq=dq, db=db, gx=gx, gy=gy, gs=gs, tol=tol, meta=meta)


# ----------------------------------------------------------------------------------------
# the five workloads (plain tiny QP, mixed-cone QCP, batched family, learned-preconditioner
# family, PSD/SOC-heavy large QCP)
# ----------------------------------------------------------------------------------------

def _kkt_active_ok(P, A, active_rows, limit=1e6):
    """Textbook QP second-order check on the generator's own active set: the KKT matrix
    [[P, A_H'], [A_H, 0]] must be well conditioned."""
    AH = A[active_rows].toarray()
    Pd = P.toarray()
    h = AH.shape[0]
    K = np.block([[Pd, AH.T], [AH, np.zeros((h, h))]])
    c = np.linalg.cond(K)
    return bool(np.isfinite(c) and c <= limit), float(c)


def tiny_qp(idx=0, max_attempts=64) -> QCP:
    """n=50, m=80 (zero 20, nonneg 60); A 80x50 density 0.1; P = BB' with B 50x5."""
    n = 50
    cones = Cones(n_zero=20, n_nonneg=60)
    for att in range(max_attempts):
        rng = np.random.default_rng([0, idx, att])
        A = sparse_gaussian(rng, cones.m, n, 0.1)
        B = rng.standard_normal((n, 5))
        P = _csr(sp.csr_matrix(np.ones((n, n))))
        Pd = B @ B.T
        Pd = 0.5 * (Pd + Pd.T)
        P.data = Pd[np.repeat(np.arange(n), n), np.tile(np.arange(n), n)].copy()
        n_act = int(rng.integers(25, 28))
        qcp = build(rng, "tiny_qp_n50_m80", n, cones, A_density=0.1, P=P, A=A,
                    nonneg_active=n_act, tol=1e-10)
        act_rows = np.concatenate([np.arange(20), 20 + np.nonzero(qcp.y[20:] > 0)[0]])
        ok, cond = _kkt_active_ok(P, A, act_rows)
        if ok:
            qcp.meta.update(seed=[0, idx, att], kkt_cond=cond)
            return qcp
    raise RuntimeError("no regular tiny QP instance found")


def mixed_qcp(idx=0) -> QCP:
    """n=5000, m=11000: zero 1000, nonneg 5000, 500 SOC(4), 10 PSD 20x20 (210 svec rows
    each), 300 exponential cones (900 rows). A density 1e-3; P = BB' + 1e-3 I with B
    5000x50 sparse (density 0.01)."""
    rng = np.random.default_rng([1, idx, 0])
    n = 5000
    cones = Cones(n_zero=1000, n_nonneg=5000, soc=[4] * 500, psd=[20] * 10, n_exp=300)
    B = sp.random(n, 50, density=0.01, random_state=rng,
                  data_rvs=rng.standard_normal, format="csr")
    P = psd_from_factor(B, 1e-3)
    psd_ranks = list(rng.integers(1, 6, size=10))
    qcp = build(rng, "mixed_qcp_n5000_m11000", n, cones, A_density=1e-3, P=P,
                nonneg_active=2000, psd_ranks=psd_ranks, tol=1e-8)
    qcp.meta["seed"] = [1, idx, 0]
    return qcp


def _face_rows_independent(qcp) -> bool:
    """The rows of A that the solution holds fixed (active nonnegative rows and every row of
    an SOC whose s is zero) are linearly independent (a plain rank test on those rows)."""
    A = qcp.A.toarray()
    c = qcp.cones
    rows = [i for i in range(c.n_zero, c.n_zero + c.n_nonneg) if qcp.s[i] == 0.0]
    r = c.n_zero + c.n_nonneg
    for k, st in zip(c.soc, qcp.meta.get("soc_states", [])):
        if st == "y_int":
            rows += list(range(r, r + k))
        r += k
    rows += list(range(c.n_zero))
    return not rows or np.linalg.matrix_rank(A[rows]) == len(rows)


def batch_member(idx=0) -> QCP:
    """One problem of the 512-problem uneven family: n ~ U{20..400}, m ~ U{1.5n..3n};
    rows PSD (k in 4..12) up to 15%, SOC (dims 3..8) up to 25%, rest nonneg; A density
    0.05; P = BB' with B n x ceil(n/10) (dense P). Face codimension aimed at 0.92 n, inside
    [0.9 n, n], so that the free directions (at most 0.1 n) do not outnumber the rank of P;
    a draw whose fixed constraint rows are linearly dependent (small n with sparse A) is
    replaced by the next draw of the same index."""
    for attempt in range(16):
        qcp = _batch_member_draw(idx, attempt)
        if _face_rows_independent(qcp):
            return qcp
    return qcp


def _batch_member_draw(idx, attempt) -> QCP:
    rng = np.random.default_rng([2, idx, attempt])
    n = int(rng.integers(20, 401))
    m_target = int(rng.integers(math.ceil(1.5 * n), math.floor(3 * n) + 1))
    psd, soc = [], []
    budget_psd = int(0.15 * m_target)
    while True:
        k = int(rng.integers(4, 13))
        if sum(kk * (kk + 1) // 2 for kk in psd) + k * (k + 1) // 2 > budget_psd:
            break
        psd.append(k)
    budget_soc = int(0.25 * m_target)
    while True:
        k = int(rng.integers(3, 9))
        if sum(soc) + k > budget_soc:
            break
        soc.append(k)
    used = sum(soc) + sum(k * (k + 1) // 2 for k in psd)
    nonneg = max(m_target - used, 1)
    cones = Cones(n_nonneg=nonneg, soc=soc, psd=psd)
    r = math.ceil(n / 10)
    B = rng.standard_normal((n, r))
    Pd = B @ B.T
    Pd = 0.5 * (Pd + Pd.T)
    P = _csr(sp.csr_matrix(np.ones((n, n))))
    P.data = Pd.reshape(-1).copy()
    target = int(round(0.92 * n))
    soc_states = [('s_int', 'y_int', 'bnd')[int(rng.integers(0, 3))] for _ in soc]
    psd_ranks = [int(rng.integers(1, max(2, k // 2 + 1))) for k in psd]

    def hard(st, k):
        return {'s_int': 0, 'y_int': k, 'bnd': 1}[st]
    cod = sum(hard(st, k) for st, k in zip(soc_states, soc)) + \
        sum(j * (j + 1) // 2 for j in psd_ranks)
    # keep the structured cones within budget, then fill with active nonneg rows
    i = 0
    while cod > target and i < len(soc):
        if soc_states[i] == 'y_int':
            soc_states[i] = 'bnd'
            cod -= soc[i] - 1
        i += 1
    n_act = int(min(max(target - cod, 0), nonneg))
    qcp = build(rng, f"batch_member_{idx}", n, cones, A_density=0.05, P=P,
                nonneg_active=n_act, soc_states=soc_states, psd_ranks=psd_ranks,
                tol=1e-8)
    qcp.meta["seed"] = [2, idx, attempt]
    return qcp


def precond_family(idx=0) -> QCP:
    """n=2000, m=4400 (zero 1100, nonneg 3300); A density 0.1; P = BB' of rank 200."""
    rng = np.random.default_rng([3, idx, 0])
    n = 2000
    cones = Cones(n_zero=1100, n_nonneg=3300)
    B = rng.standard_normal((n, 200))
    Pd = B @ B.T
    Pd = 0.5 * (Pd + Pd.T)
    P = _csr(sp.csr_matrix(np.ones((n, n))))
    P.data = Pd.reshape(-1).copy()
    n_act = int(rng.integers(760, 841))
    qcp = build(rng, f"precond_family_{idx}", n, cones, A_density=0.1, P=P,
                nonneg_active=n_act, tol=1e-8)
    qcp.meta["seed"] = [3, idx, 0]
    return qcp


def large_psd_soc(idx=0, scale=1.0) -> QCP:
    """n=20000, m=290000: nonneg 15000, 2000 SOC(10), 200 PSD 50x50 (1275 svec rows each).
    A has ~3M nnz (about 10.3 per row, N(0,1)); P = BB' with B 20000x200 at density 0.01.

    Faces: PSD rank(Y) ~ U{3..12}, SOC one third per state (s interior, y interior, boundary
    pair), and active nonnegative rows filling the hard face codimension (rows the solution
    holds fixed: active nonnegative rows, y-interior SOC rows, the j(j+1)/2 directions of a
    PSD block with rank(Y) = j, one per SOC boundary pair) to 0.8 n. The PSD cross directions
    (j(k-j) per block) and the interior directions of SOC boundary pairs add curvature, so the
    reduced Hessian is definite without the codimension reaching n - rank P; a codimension
    close to n makes the fixed rows nearly square and the derivative badly conditioned (at
    19 900 of 20 000, LSQR stalls above 1e-3).

    scale < 1 shrinks every count by that factor (PSD order and SOC dimension unchanged, same
    entries per row of A) for reduced instances of the same shape."""
    rng = np.random.default_rng([4, idx, 0])
    n = max(1, int(round(20000 * scale)))
    n_nn = int(round(15000 * scale))
    n_soc = int(round(2000 * scale))
    n_psd = max(1, int(round(200 * scale)))
    rank_p = max(1, int(round(200 * scale)))
    cones = Cones(n_nonneg=n_nn, soc=[10] * n_soc, psd=[50] * n_psd)
    m = cones.m
    B = sp.random(n, rank_p, density=0.01, random_state=rng,
                  data_rvs=rng.standard_normal, format="csr")
    P = psd_from_factor(B, 0.0)
    psd_ranks = [int(j) for j in rng.integers(3, 13, size=n_psd)]
    soc_states = [('s_int', 'y_int', 'bnd')[i % 3] for i in range(n_soc)]
    cod = sum(j * (j + 1) // 2 for j in psd_ranks) + \
        sum({'s_int': 0, 'y_int': 10, 'bnd': 1}[s] for s in soc_states)
    n_act = int(min(max(int(round(0.8 * n)) - cod, 0), n_nn))
    name = "large_psd_soc_n20000_m290000" if scale == 1.0 else f"large_psd_soc_n{n}_m{m}"
    qcp = build(rng, name, n, cones, A_density=(3.0e6 / 290000) / n, P=P,
                nonneg_active=n_act, soc_states=soc_states, psd_ranks=psd_ranks, tol=1e-8)
    qcp.meta["seed"] = [4, idx, 0]
    return qcp


def small_mixed(idx=0, n=40, n_zero=6, n_nonneg=30, soc=(3, 4, 5), psd=(2, 3, 4), n_exp=3,
                A_density=0.15, P_rank=None, P_eps=0.0, nonneg_active=None,
                psd_ranks=None, pow_alphas=(), dpow_alphas=()) -> QCP:
    """A small mixed-cone instance (every cone type) for pins and parity tests."""
    rng = np.random.default_rng([10, idx, n])
    cones = Cones(n_zero=n_zero, n_nonneg=n_nonneg, soc=list(soc), psd=list(psd),
                  n_exp=n_exp, pow=list(pow_alphas), dpow=list(dpow_alphas))
    r = P_rank if P_rank is not None else max(1, n // 4)
    B = rng.standard_normal((n, r)) / math.sqrt(r)   # P entries O(1), like A's
    Pd = B @ B.T + P_eps * np.eye(n)
    Pd = 0.5 * (Pd + Pd.T)
    P = _csr(sp.csr_matrix(np.ones((n, n))))
    P.data = Pd.reshape(-1).copy()
    if psd_ranks is None:
        psd_ranks = [max(1, k // 2) for k in psd]
    if nonneg_active is None:
        nonneg_active = n_nonneg // 3
    qcp = build(rng, f"small_mixed_{n}", n, cones, A_density=A_density, P=P,
                nonneg_active=nonneg_active, psd_ranks=psd_ranks, tol=1e-12)
    qcp.gy = rng.standard_normal(qcp.m)
    qcp.gs = rng.standard_normal(qcp.m)
    qcp.meta["seed"] = [10, idx, n]
    return qcp


CONFIGS = {
    "tiny_qp": tiny_qp,
    "mixed_qcp": mixed_qcp,
    "batch_member": batch_member,
    "precond_family": precond_family,
    "large_psd_soc": large_psd_soc,
}


def make(config: str, idx: int = 0) -> QCP:
    return CONFIGS[config](idx)
