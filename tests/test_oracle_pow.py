"""Pins of the oracle's power-cone projection and Jacobian (App. A, "Power cone", "Dual power
cone"), independent of the formulas they test:

* the projection by its variational characterisation: p_hat = Pi_K(p) exactly when p_hat is
  in K, <p_hat, p - p_hat> = 0 and <p - p_hat, q> <= 0 for every q in K (p - p_hat in the
  polar cone), the last checked on the cone's extreme rays, densely sampled;
* the closed-form Jacobian against central differences of the projection, on random points
  of every case (interior, polar interior, the z = 0 case with both signs of x and y and the
  three regimes of alpha, and the root-finding case);
* symmetry, spectrum in [0, 1] and Euler's identity J p = Pi(p) (the projection is
  positively homogeneous);
* the dual cone through Moreau (Pi_{K*}(v) = v + Pi_K(-v)) checked against K* directly;
* planted mistakes in the closed form fail the difference check.
"""
import math

import numpy as np
import pytest

from oracle import cones as C

ALPHAS = (0.2, 0.5, 0.7, 0.9)


# Membership up to rounding, as a distance: the point moved by d (a small multiple of the
# rounding unit times the scale) along (1, 1, 0) must lie in the cone. A plain test of
# x^a y^(1-a) >= |z| at the point itself is far more sensitive than the point: near the face
# y = 0 the product moves by up to 1e-6 relative when y moves by one unit in its last place.
def pow_ok(p, a, d):
    x, y, z = p
    return x >= -d and y >= -d and \
        max(x + d, 0) ** a * max(y + d, 0) ** (1 - a) >= abs(z)


def dual_ok(p, a, d):
    u, v, w = p
    return u >= -d and v >= -d and \
        (max(u + d, 0) / a) ** a * (max(v + d, 0) / (1 - a)) ** (1 - a) >= abs(w)


THETA = np.concatenate([np.geomspace(1e-16, 1e-3, 400), np.linspace(1e-3, math.pi / 2 - 1e-3, 2000),
                        math.pi / 2 - np.geomspace(1e-16, 1e-3, 400)])


def rays(a, dual=False):
    """Unit-ish generators of the boundary of K (or K*): (c, s, +-c^a s^(1-a)) with
    (c, s) = (cos t, sin t), resp. (c, s, +-(c/a)^a (s/(1-a))^(1-a))."""
    c, s = np.cos(THETA), np.sin(THETA)
    h = (c / a) ** a * (s / (1 - a)) ** (1 - a) if dual else c ** a * s ** (1 - a)
    return np.concatenate([np.stack([c, s, h], 1), np.stack([c, s, -h], 1)])


def polar_violation(d, a, dual=False):
    """max over generators q of the cone of <d, q> (<= 0 when d is in the polar cone)."""
    return float((rays(a, dual) @ d).max())


def points(rng, count):
    for _ in range(count):
        yield rng.standard_normal(3) * rng.uniform(0.05, 6.0)


@pytest.mark.parametrize("a", ALPHAS)
def test_projection_moreau(a):
    rng = np.random.default_rng(int(a * 100))
    for p in points(rng, 400):
        ph = C.proj_pow(p, a)
        sc = 1.0 + np.abs(p).max()
        assert pow_ok(ph, a, 1e-14 * sc), (p, ph)
        assert polar_violation(p - ph, a) <= 1e-12 * sc, (p, ph)
        assert abs(ph @ (p - ph)) <= 1e-12 * sc * sc


@pytest.mark.parametrize("a", ALPHAS)
def test_dual_projection_moreau(a):
    rng = np.random.default_rng(7 + int(a * 100))
    for v in points(rng, 300):
        vh = C.proj_pow_dual(v, a)
        sc = 1.0 + np.abs(v).max()
        assert dual_ok(vh, a, 1e-14 * sc)
        assert polar_violation(v - vh, a, dual=True) <= 1e-12 * sc
        assert abs(vh @ (v - vh)) <= 1e-12 * sc * sc


def fd_jac(f, p, h):
    return np.stack([(f(p + h * e) - f(p - h * e)) / (2 * h) for e in np.eye(3)], axis=1)


def case_points(a, rng):
    """Points of every case of the appendix's list."""
    out = []
    for p in points(rng, 200):
        out.append(p)
    # the z = 0 case, x and y of opposite signs
    for _ in range(20):
        x, y = rng.uniform(0.2, 3.0), -rng.uniform(0.2, 3.0)
        out.append(np.array([x, y, 0.0]))
        out.append(np.array([y, x, 0.0]))
    # close to the boundary of K from outside (the root lies near |z|)
    for _ in range(20):
        x, y = rng.uniform(0.2, 3.0, size=2)
        out.append(np.array([x, y, (1.0 + rng.uniform(0.01, 0.3)) * x ** a * y ** (1 - a)]))
    return out


@pytest.mark.parametrize("a", ALPHAS)
def test_jacobian_against_differences(a):
    rng = np.random.default_rng(100 + int(a * 100))
    worst = 0.0
    for p in case_points(a, rng):
        sc = 1.0 + np.abs(p).max()
        J = C.jac_pow(p, a)
        # at z = 0 the projection is differentiable but its z-derivative is approached with
        # an error like a power of |z| below 2: a smaller step there
        h = (1e-9 if p[2] == 0.0 else 1e-6) * sc
        Jfd = fd_jac(lambda q: C.proj_pow(q, a), p, h)
        worst = max(worst, np.abs(J - Jfd).max())
        assert np.abs(J - Jfd).max() <= 1e-6, (p, J, Jfd)
        assert np.abs(J - J.T).max() <= 1e-12
        ev = np.linalg.eigvalsh(0.5 * (J + J.T))
        assert ev.min() >= -1e-10 and ev.max() <= 1 + 1e-10
        assert np.abs(J @ p - C.proj_pow(p, a)).max() <= 1e-10 * sc
    print(f"alpha {a}: worst |J - FD| {worst:.1e}")


def test_z_zero_alpha_half_matches_dx_dy():
    """At z = 0, alpha = 1/2, the z-derivative of the projection (by differences through the
    z != 0 case on both sides) is x / (2|y| + x) for x > 0 > y and y / (2|x| + y) for
    y > 0 > x."""
    for x, y in ((1.3, -0.4), (0.2, -2.0), (-0.7, 1.1), (-3.0, 0.25)):
        p = np.array([x, y, 0.0])
        h = 1e-7
        dz = (C.proj_pow(p + [0, 0, h], 0.5)[2] - C.proj_pow(p - [0, 0, h], 0.5)[2]) / (2 * h)
        expect = x / (2 * abs(y) + x) if x > 0 else y / (2 * abs(x) + y)
        assert abs(dz - expect) <= 1e-6, (x, y, dz, expect)
        assert abs(C.jac_pow(p, 0.5)[2, 2] - expect) <= 1e-15


@pytest.mark.parametrize("a", (0.3, 0.8))
def test_z_zero_other_alphas(a):
    """Away from alpha = 1/2 the z-derivative at z = 0 is 0 or 1 by which of x, y is
    positive (the larger exponent wins)."""
    for x, y in ((1.3, -0.4), (-0.7, 1.1)):
        p = np.array([x, y, 0.0])
        h = 1e-8
        dz = (C.proj_pow(p + [0, 0, h], a)[2] - C.proj_pow(p - [0, 0, h], a)[2]) / (2 * h)
        assert abs(dz - C.jac_pow(p, a)[2, 2]) <= 1e-5, (a, x, y, dz)


def test_dual_jacobian_by_differences():
    rng = np.random.default_rng(5)
    for a in ALPHAS:
        for v in points(rng, 60):
            sc = 1.0 + np.abs(v).max()
            J = C.jac_pow_dual(v, a)
            Jfd = fd_jac(lambda q: C.proj_pow_dual(q, a), v, 1e-6 * sc)
            assert np.abs(J - Jfd).max() <= 1e-6


@pytest.mark.parametrize("mistake", ["sign_xz", "L_inverted", "T_sign"])
def test_planted_mistakes_fail(mistake, monkeypatch):
    """A wrong sign of the (x, z) entry, L replaced by 1/L, or T with the wrong sign each fail
    the difference check on root-finding points."""
    real = C.jac_pow

    def wrong(p, a):
        J = real(p, a).copy()
        x, y, z = p
        if C.in_pow(p, a) or C.in_pow_polar(p, a) or z == 0.0:
            return J
        r = C._pow_root(p, a)
        fx, fy = C._pow_f(x, y, z, a, r)
        az = abs(z)
        gx, gy = 2 * fx - x, 2 * fy - y
        S = a * x / gx + (1 - a) * y / gy
        L = 2 * (az - r) / (az + (az - 2 * r) * S)
        if mistake == "sign_xz":
            J[0, 2] = J[2, 0] = -J[0, 2]
        elif mistake == "L_inverted":
            J[2, 2] = r / az + (r / az) * (-S) / L
        else:
            J[2, 2] = r / az + (r / az) * S * L
        return J

    monkeypatch.setattr(C, "jac_pow", wrong)
    rng = np.random.default_rng(11)
    bad = 0
    for p in points(rng, 200):
        if C.in_pow(p, 0.3) or C.in_pow_polar(p, 0.3) or p[2] == 0.0:
            continue
        sc = 1.0 + np.abs(p).max()
        Jfd = fd_jac(lambda q: C.proj_pow(q, 0.3), p, 1e-6 * sc)
        bad += np.abs(C.jac_pow(p, 0.3) - Jfd).max() > 1e-6
    assert bad > 0


# ---- the derivative of a program with power cones ---------------------------------------

def pow_instance():
    import qcpgen
    return qcpgen.small_mixed(5, n=40, pow_alphas=(0.3, 0.5, 0.8), dpow_alphas=(0.25, 0.6, 0.5),
                              P_eps=0.1)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_generated_pairs_are_complementary():
    """The generator's pairs: s in the cone, y in its dual, s'y = 0 per block, so that the
    projection of y - s onto the dual cone returns y."""
    q = pow_instance()
    r = q.m - 3 * (len(q.cones.pow) + len(q.cones.dpow))
    for i, a in enumerate(list(q.cones.pow) + list(q.cones.dpow)):
        s, y = q.s[r + 3 * i:r + 3 * i + 3], q.y[r + 3 * i:r + 3 * i + 3]
        dual = i >= len(q.cones.pow)
        assert (dual_ok(s, a, 1e-14) if dual else pow_ok(s, a, 1e-14))
        assert (pow_ok(y, a, 1e-14) if dual else dual_ok(y, a, 1e-14))
        assert abs(s @ y) <= 1e-14
    assert np.abs(C.proj_dual(q.y - q.s, q.cones) - q.y).max() <= 1e-14


def test_jvp_with_power_cones_matches_newton_differences():
    """Central differences of a semismooth Newton re-solve (values only) against the JVP, and
    the dense implicit-function solve against the paper's least-squares steps."""
    from oracle import derivative as D
    from oracle import embedding as E
    q = pow_instance()
    got = D.jvp(q, q.dP, q.dA, q.dq, q.db, tol=1e-13)
    h = 1e-6
    qp = E.with_data(q, q.dP, q.dA, q.dq, q.db, h=h)
    qm = E.with_data(q, q.dP, q.dA, q.dq, q.db, h=-h)
    xp, yp, sp_, rp = D.newton_resolve(qp, q.x, q.y - q.s)
    xm, ym, sm, rm = D.newton_resolve(qm, q.x, q.y - q.s)
    assert rp < 1e-13 and rm < 1e-13
    fd = ((xp - xm) / (2 * h), (yp - ym) / (2 * h), (sp_ - sm) / (2 * h))
    for a, b in zip(got, fd):
        assert rel(a, b) < 1e-6
    for a, b in zip(got, D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)):
        assert rel(a, b) < 1e-9


def test_vjp_with_power_cones_adjoint_identity():
    from oracle import derivative as D
    q = pow_instance()
    dx, dy, ds = D.jvp(q, q.dP, q.dA, q.dq, q.db, tol=1e-13)
    dP, dA, dq, db = D.vjp(q, q.gx, q.gy, q.gs, tol=1e-13)
    lhs = q.gx @ dx + q.gy @ dy + q.gs @ ds
    rhs = dP @ q.dP + dA @ q.dA + dq @ q.dq + db @ q.db
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)
