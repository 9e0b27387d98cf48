"""Pins for the oracle's cone projections and Jacobians (Appendix A).

Projections are pinned by Moreau's characterisation (Sec. 2.3, "Other machinery":
Pi_K(v) + Pi_{K polar}(v) = v): p = Pi_K(v) iff p in K, v - p in K polar, <p, v - p> = 0.
Jacobians are pinned by central finite differences of the pinned projections, symmetry,
spectrum in [0, 1], and Euler's identity J(z) z = Pi(z) (projections onto cones are
positively homogeneous). Special cases reduce to simpler cones; two hand-worked examples
live under tests/golden/.
"""
import math
import os

import numpy as np
import pytest

import qcpgen
from oracle import cones as C

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        out[parts[0]] = np.array([float(t) for t in parts[1:]])
    return out


def _fd_jac(f, z, h=1e-6):
    k = z.size
    J = np.empty((k, k))
    for c in range(k):
        e = np.zeros(k)
        e[c] = h
        J[:, c] = (f(z + e) - f(z - e)) / (2 * h)
    return J


# ---- membership tests used by the Moreau pins ---------------------------------------

def in_soc(p, tol):
    return np.linalg.norm(p[1:]) <= p[0] + tol


def in_psd(v, tol):
    k = C.psd_order(v.size)
    return np.linalg.eigvalsh(C.smat(v, k)).min() >= -tol


def in_exp_tol(p, tol):
    x, y, z = p
    if y > tol:
        return y * math.exp(min(x / y, 700)) <= z + tol * (1 + abs(z))
    return abs(y) <= tol and x <= tol and z >= -tol


def in_exp_dual_tol(p, tol):
    u, v, w = p
    if u < -tol:
        return -u * math.exp(min(v / u, 700)) <= math.e * w + tol * (1 + abs(w))
    return abs(u) <= tol and v >= -tol and w >= -tol


# ---- nonnegative ------------------------------------------------------------------------

def test_nonneg_moreau():
    rng = np.random.default_rng(0)
    v = rng.standard_normal(1000)
    p = C.proj_nonneg(v)
    r = v - p
    assert (p >= 0).all() and (r <= 0).all() and abs(p @ r) == 0.0


def test_nonneg_jacobian_fd():
    rng = np.random.default_rng(1)
    v = rng.standard_normal(50)
    v[np.abs(v) < 1e-3] = 0.5
    J = np.diag(C.jac_nonneg_diag(v))
    assert np.allclose(J, _fd_jac(C.proj_nonneg, v), atol=1e-9)


# ---- second-order cone ------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2, 3, 5, 10])
def test_soc_moreau(k):
    rng = np.random.default_rng(k)
    for _ in range(200):
        v = rng.standard_normal(k) * rng.uniform(0.1, 10)
        p = C.proj_soc(v)
        r = v - p
        sc = 1e-12 * (1 + np.linalg.norm(v))
        assert in_soc(p, sc)
        assert in_soc(-r, sc)        # polar of a self-dual cone is its negative
        assert abs(p @ r) <= sc * (1 + np.linalg.norm(v))


def test_soc_dim1_is_nonneg():
    for t in (-2.0, -1e-3, 0.0, 0.7, 3.0):
        assert C.proj_soc(np.array([t]))[0] == max(t, 0.0)


def test_soc_golden():
    g = _read_golden("soc_3.txt")
    assert np.allclose(C.proj_soc(g["z"]), g["proj"], atol=1e-15)
    J = np.stack([g["J_row0"], g["J_row1"], g["J_row2"]])
    assert np.allclose(C.jac_soc(g["z"]), J, atol=1e-15)


@pytest.mark.parametrize("k", [2, 3, 4, 8])
def test_soc_jacobian_fd_and_structure(k):
    rng = np.random.default_rng(10 + k)
    for case in range(30):
        z = rng.standard_normal(k) * 2
        nu = np.linalg.norm(z[1:])
        if abs(nu - abs(z[0])) < 1e-2:
            continue
        J = C.jac_soc(z)
        assert np.allclose(J, _fd_jac(C.proj_soc, z), atol=1e-7)
        assert np.allclose(J, J.T, atol=1e-14)
        ev = np.linalg.eigvalsh(J)
        assert ev.min() >= -1e-12 and ev.max() <= 1 + 1e-12
        assert np.allclose(J @ z, C.proj_soc(z), atol=1e-12)


# ---- PSD ----------------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2, 3, 6, 12])
def test_psd_moreau(k):
    rng = np.random.default_rng(20 + k)
    for _ in range(20):
        G = rng.standard_normal((k, k))
        v = C.svec(G + G.T)
        p = C.proj_psd(v)
        r = v - p
        assert in_psd(p, 1e-12)
        assert in_psd(-r, 1e-12)
        assert abs(p @ r) <= 1e-12 * (1 + v @ v)


def test_psd_special_cases():
    # 1x1 PSD block is the nonnegative cone
    for t in (-1.5, 0.0, 2.5):
        assert C.proj_psd(np.array([t]))[0] == pytest.approx(max(t, 0.0), abs=1e-15)
    # a diagonal matrix projects by clipping its diagonal
    d = np.array([3.0, -1.0, 0.5, -2.0])
    p = C.proj_psd(C.svec(np.diag(d)))
    assert np.allclose(C.smat(p, 4), np.diag(np.maximum(d, 0)), atol=1e-14)


def test_psd_golden():
    g = _read_golden("psd_2x2.txt")
    assert np.allclose(C.proj_psd(g["z"]), g["proj"], atol=1e-15)
    J = np.stack([g["J_row0"], g["J_row1"], g["J_row2"]])
    assert np.allclose(C.jac_psd(g["z"]), J, atol=1e-15)


@pytest.mark.parametrize("k", [2, 3, 5, 8])
def test_psd_jacobian_fd_and_structure(k):
    rng = np.random.default_rng(40 + k)
    for _ in range(5):
        U = qcpgen.random_orthogonal(rng, k)
        lam = rng.uniform(0.2, 2, size=k) * rng.choice([-1, 1], size=k)
        z = C.svec((U * lam) @ U.T)
        J = C.jac_psd(z)
        assert np.allclose(J, _fd_jac(C.proj_psd, z), atol=1e-7)
        assert np.allclose(J, J.T, atol=1e-13)
        ev = np.linalg.eigvalsh(J)
        assert ev.min() >= -1e-12 and ev.max() <= 1 + 1e-12
        assert np.allclose(J @ z, C.proj_psd(z), atol=1e-12)


def test_psd_all_nonneg_or_all_negative():
    rng = np.random.default_rng(3)
    U = qcpgen.random_orthogonal(rng, 4)
    zp = C.svec((U * np.array([1, 2, 0.5, 3.0])) @ U.T)
    zn = -zp
    assert np.allclose(C.jac_psd(zp), np.eye(10), atol=1e-13)
    assert np.allclose(C.jac_psd(zn), 0.0, atol=1e-13)


def test_psd_diagonal_estimate_matches_dense():
    rng = np.random.default_rng(5)
    U = qcpgen.random_orthogonal(rng, 5)
    lam = np.array([1.0, -0.5, 0.3, -2.0, 0.7])
    z = C.svec((U * lam) @ U.T)
    cones = qcpgen.Cones(psd=[5])
    Jo = C.DualJacobian(z, cones)
    assert np.allclose(Jo.diagonal(), np.diag(C.jac_psd(z)), atol=1e-13)


# ---- exponential ----------------------------------------------------------------------------

def _exp_points(rng, count):
    pts = []
    for _ in range(count):
        pts.append(rng.standard_normal(3) * rng.uniform(0.2, 3))
    return pts


def test_exp_moreau_random():
    rng = np.random.default_rng(7)
    for v in _exp_points(rng, 300):
        p = C.proj_exp(v)
        r = v - p
        tol = 1e-10 * (1 + np.linalg.norm(v))
        assert in_exp_tol(p, tol), (v, p)
        assert in_exp_dual_tol(-r, tol), (v, r)   # r in polar = -K*
        assert abs(p @ r) <= tol, (v, p, r)


def test_exp_known_complementary_pairs():
    """Pi_exp(s - y) = s for s in K_exp, y in K_exp*, s'y = 0 (Moreau)."""
    rng = np.random.default_rng(8)
    for st in ("s_int", "y_int", "bnd") * 30:
        s, y, _, _ = qcpgen._exp_pair(rng, st)
        assert abs(s @ y) < 1e-14
        assert np.allclose(C.proj_exp(s - y), s, atol=1e-12)
        # and the dual-cone projection used by the embedding returns y
        assert np.allclose(C.proj_exp_dual(y - s), y, atol=1e-12)


def test_exp_jacobian_fd():
    rng = np.random.default_rng(9)
    n_case4 = 0
    for st in ("s_int", "y_int", "bnd") * 10:
        s, y, _, _ = qcpgen._exp_pair(rng, st)
        p = s - y
        J = C.jac_exp(p)
        Jfd = _fd_jac(C.proj_exp, p, h=1e-6)
        assert np.allclose(J, Jfd, atol=2e-7), (st, J, Jfd)
        ev = np.linalg.eigvalsh(0.5 * (J + J.T))
        assert ev.min() >= -1e-10 and ev.max() <= 1 + 1e-10
        assert np.allclose(J @ p, C.proj_exp(p), atol=1e-10)
        n_case4 += st == "bnd"
    assert n_case4 == 10


def test_exp_jacobian_region_cases():
    # interior of K -> I, interior of polar -> 0, x<0,y<0 -> diag(1,0,1{z>0})
    assert np.allclose(C.jac_exp(np.array([-1.0, 1.0, 5.0])), np.eye(3))
    assert np.allclose(C.jac_exp(-np.array([-1.0, 0.5, 5.0])), 0.0)
    assert np.allclose(C.jac_exp(np.array([-1.0, -2.0, 3.0])), np.diag([1.0, 0.0, 1.0]))
    assert np.allclose(C.jac_exp(np.array([-1.0, -2.0, -3.0])), np.diag([1.0, 0.0, 0.0]))
    # the third closed case of the projection
    assert np.allclose(C.proj_exp(np.array([-1.0, -2.0, 3.0])), [-1.0, 0.0, 3.0])


def test_exp_entry22_sign_reading():
    """The printed (2,2) entry '1 + -mu x^2 e^{x/y}/y^3' is read with '+'; the '-' reading
    disagrees with finite differences. Planting the '-' reading must fail the FD pin."""
    rng = np.random.default_rng(11)
    s, y, _, prm = qcpgen._exp_pair(rng, "bnd")
    p = s - y
    phat, r, yhat, mu = C._exp_case4(p)
    xs, ys = phat[0], phat[1]
    e = math.exp(xs / ys)
    J4 = np.array([
        [1 + mu * e / ys, -mu * xs * e / ys ** 2, 0.0, e],
        [-mu * xs * e / ys ** 2, 1 - mu * xs ** 2 * e / ys ** 3, 0.0, (1 - xs / ys) * e],
        [0.0, 0.0, 1.0, -1.0],
        [e, (1 - xs / ys) * e, -1.0, 0.0]])
    wrong = np.linalg.inv(J4)[:3, :3]
    Jfd = _fd_jac(C.proj_exp, p)
    assert not np.allclose(wrong, Jfd, atol=1e-4) or abs(xs) < 1e-3
    assert np.allclose(C.jac_exp(p), Jfd, atol=2e-7)
    # the generator's parameters are recovered: r, yhat, mu
    assert r == pytest.approx(prm["r"], abs=1e-10)
    assert yhat == pytest.approx(prm["s2"], rel=1e-10)
    assert mu == pytest.approx(prm["mu"], rel=1e-10)


def test_dual_jacobian_blocks_match_single_cone_functions():
    q = qcpgen.small_mixed(0)
    z = q.y - q.s
    Jo = C.DualJacobian(z, q.cones)
    Jd = Jo.dense_matrix()
    f = lambda v: C.proj_dual(v, q.cones)
    # away from kinks the whole block-diagonal J matches FD of the product projection
    assert np.allclose(Jd, _fd_jac(f, z), atol=2e-7)
    assert np.allclose(Jd, Jd.T, atol=1e-12)
    assert np.allclose(Jo.diagonal(), np.diag(Jd), atol=1e-13)
