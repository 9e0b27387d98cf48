"""Pins for the oracle's embedding algebra (Sec. 2.1 - 2.4).

* The generator's solutions satisfy the KKT conditions and R(z) = 0 (eq. residual-map).
* F = D_z N against central differences of N (eq. normalized-residual).
* F z = 0: R is positively homogeneous (Sec. 2.3), so its derivative annihilates z.
* <r, F v> = <F' r, v> (adjoint pair).
* D_theta N against differences in theta (N is affine in theta, so they are exact).
* D_theta N' against D_theta N through the inner product on stored entries.
* D phi against differences of phi; D phi z = 0 (phi is homogeneous of degree 0).
Mutations planted in the oracle (a dropped term, a sign, a transpose) must break a pin.
"""
import numpy as np
import pytest

import qcpgen
from oracle import embedding as E


@pytest.fixture(scope="module", params=["tiny", "mixed"])
def inst(request):
    if request.param == "tiny":
        return qcpgen.tiny_qp(0)
    return qcpgen.small_mixed(0)


def test_kkt_and_residual_zero(inst):
    q = inst
    assert np.linalg.norm(q.A @ q.x + q.s - q.b) < 1e-12 * (1 + np.linalg.norm(q.b))
    assert np.linalg.norm(q.P @ q.x + q.A.T @ q.y + q.q) < 1e-12 * (1 + np.linalg.norm(q.q))
    assert abs(q.s @ q.y) < 1e-12
    z = E.point_from_solution(q.x, q.y, q.s)
    assert np.linalg.norm(E.residual(q, z)) < 1e-12 * (1 + np.linalg.norm(q.q) + np.linalg.norm(q.b))


def test_F_matches_finite_differences(inst):
    q = inst
    emb = E.Embedding(q)
    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(3):
        v = rng.standard_normal(emb.N)
        fd = (E.normalized_residual(q, emb.z + h * v) - E.normalized_residual(q, emb.z - h * v)) / (2 * h)
        assert np.linalg.norm(emb.F(v) - fd) <= 1e-7 * np.linalg.norm(fd)


def test_F_annihilates_z(inst):
    emb = E.Embedding(inst)
    assert np.linalg.norm(emb.F(emb.z)) <= 1e-12 * np.linalg.norm(emb.z) * 10


def test_F_adjoint_pair(inst):
    emb = E.Embedding(inst)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(emb.N)
    r = rng.standard_normal(emb.N)
    a, b = r @ emb.F(v), emb.FT(r) @ v
    assert abs(a - b) <= 1e-12 * (abs(a) + np.linalg.norm(r) * np.linalg.norm(v))


def test_dtheta_exact_differences(inst):
    q = inst
    emb = E.Embedding(q)
    h = 1e-3
    qp = E.with_data(q, q.dP, q.dA, q.dq, q.db, h=h)
    qm = E.with_data(q, q.dP, q.dA, q.dq, q.db, h=-h)
    fd = (E.normalized_residual(qp, emb.z) - E.normalized_residual(qm, emb.z)) / (2 * h)
    got = emb.dtheta(q.dP, q.dA, q.dq, q.db)
    assert np.linalg.norm(got - fd) <= 1e-9 * np.linalg.norm(fd)


def test_dtheta_adjoint_on_patterns(inst):
    q = inst
    emb = E.Embedding(q)
    rng = np.random.default_rng(2)
    w = rng.standard_normal(emb.N)
    dP, dA, dq, db = emb.dtheta_t(w)
    lhs = w @ emb.dtheta(q.dP, q.dA, q.dq, q.db)
    rhs = dP @ q.dP + dA @ q.dA + dq @ q.dq + db @ q.db
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    # the returned dP is symmetric on the pattern
    t = qcpgen.transpose_slots(q.P)
    assert np.allclose(dP, dP[t], rtol=1e-15, atol=1e-15)


def test_dphi_differences_and_homogeneity(inst):
    q = inst
    emb = E.Embedding(q)
    rng = np.random.default_rng(3)
    h = 1e-6
    v = rng.standard_normal(emb.N)
    fp = E.phi(q, emb.z + h * v)
    fm = E.phi(q, emb.z - h * v)
    got = emb.dphi(v)
    for a, p_, m_ in zip(got, fp, fm):
        fd = (p_ - m_) / (2 * h)
        assert np.linalg.norm(a - fd) <= 1e-7 * (1 + np.linalg.norm(fd))
    for part in emb.dphi(emb.z):
        assert np.linalg.norm(part) <= 1e-12 * np.linalg.norm(emb.z)
    # D phi' is the adjoint of D phi
    gx = rng.standard_normal(q.n)
    gy = rng.standard_normal(q.m)
    gs = rng.standard_normal(q.m)
    lhs = gx @ got[0] + gy @ got[1] + gs @ got[2]
    rhs = emb.dphi_t(gx, gy, gs) @ v
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(v) * 10)


# ---- planted mistakes must be caught ----------------------------------------------------

def _F_pin_holds(q, emb):
    rng = np.random.default_rng(0)
    h = 1e-6
    v = rng.standard_normal(emb.N)
    fd = (E.normalized_residual(q, emb.z + h * v) - E.normalized_residual(q, emb.z - h * v)) / (2 * h)
    return np.linalg.norm(emb.F(v) - fd) <= 1e-7 * np.linalg.norm(fd)


def test_planted_sign_error_in_tau_row_is_caught(monkeypatch):
    q = qcpgen.small_mixed(0)
    emb = E.Embedding(q)
    assert _F_pin_holds(q, emb)
    orig = E.Embedding.dq

    def bad(self, w):
        out = orig(self, w)
        out[-1] += 2 * (self.qcp.q @ w[:self.n])   # flips the sign of the -q'w_x term
        return out
    monkeypatch.setattr(E.Embedding, "dq", bad)
    assert not _F_pin_holds(q, emb)


def test_planted_transpose_error_is_caught(monkeypatch):
    q = qcpgen.small_mixed(0)
    emb = E.Embedding(q)
    orig = E.Embedding.dq_t

    def bad(self, r):
        out = orig(self, r)
        n, m = self.n, self.m
        # use +A'r_y instead of -A'r_y in the x rows
        out[:n] += 2 * (self.qcp.A.T @ r[n:n + m])
        return out
    monkeypatch.setattr(E.Embedding, "dq_t", bad)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(emb.N)
    r = rng.standard_normal(emb.N)
    assert abs(r @ emb.F(v) - emb.FT(r) @ v) > 1e-6
