"""Pins for the oracle's LSQR and its JVP / VJP (Sec. 3.1, 3.2).

* LSQR against SciPy's lsqr (library) and exact solutions.
* JVP of a zero/nonnegative QP against the textbook active-set KKT derivative.
* JVP of a mixed-cone instance against central differences of a Newton re-solve (values
  only define that root) and against the dense reduced-KKT implicit-function solve.
* VJP against the adjoint identity <g, JVP(dtheta)> = <VJP(g), dtheta> (inner product
  over stored entries for dP and dA) and against the dense adjoint solve.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import qcpgen
from oracle import derivative as D
from oracle import embedding as E
from oracle.lsqr import lsqr


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ---- LSQR --------------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(40, 25), (25, 40), (30, 30)])
def test_lsqr_matches_scipy(shape):
    rng = np.random.default_rng(shape[0])
    A = rng.standard_normal(shape)
    b = rng.standard_normal(shape[0])
    x, info = lsqr(lambda v: A @ v, lambda u: A.T @ u, b, tol=1e-14, max_iter=2000)
    ref = spla.lsqr(A, b, atol=0, btol=1e-14, iter_lim=2000)[0]
    assert rel(x, ref) < 1e-9
    # least-squares optimality: A'(b - Ax) = 0
    assert np.linalg.norm(A.T @ (b - A @ x)) < 1e-9 * np.linalg.norm(A) * np.linalg.norm(b)


def test_lsqr_column_scaling_keeps_solution_of_consistent_system():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((30, 30))
    xs = rng.standard_normal(30)
    b = A @ xs
    d = rng.uniform(0.1, 10, size=30)
    x, info = lsqr(lambda v: A @ v, lambda u: A.T @ u, b, tol=1e-14, col_scale=d)
    assert info["converged"] and rel(x, xs) < 1e-8


def test_lsqr_zero_rhs():
    A = np.eye(3)
    x, info = lsqr(lambda v: A @ v, lambda u: A.T @ u, np.zeros(3))
    assert np.all(x == 0) and info["iters"] == 0


# ---- JVP ---------------------------------------------------------------------------------

@pytest.mark.parametrize("idx", [0, 1, 2])
def test_tiny_qp_jvp_matches_textbook_active_set(idx):
    q = qcpgen.tiny_qp(idx)
    got = D.jvp(q, q.dP, q.dA, q.dq, q.db, tol=1e-13)
    ref = D.qp_active_set_jvp(q, q.dP, q.dA, q.dq, q.db)
    for a, b in zip(got, ref):
        assert rel(a, b) < 1e-8


def test_dense_ift_matches_textbook_active_set():
    q = qcpgen.tiny_qp(0)
    got = D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)
    ref = D.qp_active_set_jvp(q, q.dP, q.dA, q.dq, q.db)
    for a, b in zip(got, ref):
        assert rel(a, b) < 1e-11


@pytest.fixture(scope="module")
def mixed():
    q = qcpgen.small_mixed(0)
    emb = E.Embedding(q)
    return q, emb


def test_mixed_jvp_matches_newton_finite_differences(mixed):
    q, emb = mixed
    got = D.jvp(q, q.dP, q.dA, q.dq, q.db, tol=1e-13, emb=emb)
    h = 1e-6
    qp = E.with_data(q, q.dP, q.dA, q.dq, q.db, h=h)
    qm = E.with_data(q, q.dP, q.dA, q.dq, q.db, h=-h)
    xp, yp, sp_, rp = D.newton_resolve(qp, q.x, q.y - q.s)
    xm, ym, sm, rm = D.newton_resolve(qm, q.x, q.y - q.s)
    assert rp < 1e-13 and rm < 1e-13
    fd = ((xp - xm) / (2 * h), (yp - ym) / (2 * h), (sp_ - sm) / (2 * h))
    for a, b in zip(got, fd):
        assert rel(a, b) < 1e-6


def test_mixed_jvp_matches_dense_ift(mixed):
    q, emb = mixed
    got = D.jvp(q, q.dP, q.dA, q.dq, q.db, tol=1e-13, emb=emb)
    ref = D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)
    for a, b in zip(got, ref):
        assert rel(a, b) < 1e-9


def test_mixed_jvp_unpreconditioned_agrees(mixed):
    q, emb = mixed
    a = D.jvp(q, q.dP, q.dA, q.dq, q.db, tol=1e-13, emb=emb, precond=None)
    b = D.jvp(q, q.dP, q.dA, q.dq, q.db, tol=1e-13, emb=emb)
    for u, v in zip(a, b):
        assert rel(u, v) < 1e-9


# ---- VJP ---------------------------------------------------------------------------------

def test_mixed_vjp_adjoint_identity_and_dense(mixed):
    q, emb = mixed
    dx, dy, ds = D.jvp(q, q.dP, q.dA, q.dq, q.db, tol=1e-13, emb=emb)
    dP, dA, dq, db = D.vjp(q, q.gx, q.gy, q.gs, tol=1e-13, emb=emb)
    lhs = q.gx @ dx + q.gy @ dy + q.gs @ ds
    rhs = dP @ q.dP + dA @ q.dA + dq @ q.dq + db @ q.db
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)
    ref = D.vjp_dense(q, q.gx, q.gy, q.gs)
    for a, b in zip((dP, dA, dq, db), ref):
        assert rel(a, b) < 1e-9


def test_tiny_vjp_adjoint_identity():
    q = qcpgen.tiny_qp(1)
    dx, dy, ds = D.jvp(q, q.dP, q.dA, q.dq, q.db, tol=1e-13)
    dP, dA, dq, db = D.vjp(q, q.gx, q.gy, q.gs, tol=1e-13)
    lhs = q.gx @ dx + q.gy @ dy + q.gs @ ds
    rhs = dP @ q.dP + dA @ q.dA + dq @ q.dq + db @ q.db
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)


def test_planted_dphi_error_is_caught(monkeypatch):
    """Dropping the -dz_N * x term of D phi must break the textbook-QP pin."""
    q = qcpgen.tiny_qp(0)
    orig = E.Embedding.dphi

    def bad(self, dz):
        dx, dy, ds = orig(self, dz)
        return dx + dz[-1] * self.u[:self.n], dy, ds
    monkeypatch.setattr(E.Embedding, "dphi", bad)
    got = D.jvp(q, q.dP, q.dA, q.dq, q.db, tol=1e-13)
    ref = D.qp_active_set_jvp(q, q.dP, q.dA, q.dq, q.db)
    assert rel(got[0], ref[0]) > 1e-6


def test_shared_factorisation_equals_separate_dense_solves():
    """jvp_vjp_dense (one LU for both directions, A'J from the sparse A) gives the same
    numbers as jvp_dense and vjp_dense, which the other pins of this file anchor."""
    q = qcpgen.small_mixed(1, n=120, A_density=0.08, P_rank=100, P_eps=0.1)
    assert D.kred_cond(q) < 1e8
    (dx, dy, ds), (dP, dA, dq, db) = D.jvp_vjp_dense(q, q.dP, q.dA, q.dq, q.db, q.gx, q.gy, q.gs)
    for a, r in zip((dx, dy, ds), D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)):
        assert rel(a, r) < 1e-12
    for a, r in zip((dP, dA, dq, db), D.vjp_dense(q, q.gx, q.gy, q.gs)):
        assert rel(a, r) < 1e-12
