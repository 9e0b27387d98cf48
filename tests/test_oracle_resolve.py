"""Pins of the oracle's forward re-solve (derivative.newton_resolve), the reference of the
library's refinement: from a perturbed point of an unchanged instance it returns the
instance's known solution (the generator builds the data around it); the KKT map it drives
to zero vanishes at that solution and is of the order of the perturbation away from it; the
returned y and s lie in K* and K (y = Pi_{K*}(y - s) and Pi_K(s) = s) with y's = 0."""
import numpy as np
import pytest

import qcpgen
from oracle import cones as C
from oracle import derivative as D


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1.0)


@pytest.fixture(scope="module")
def inst():
    rng = np.random.default_rng([31, 2])
    return qcpgen.small_mixed(2, n=60, n_zero=6, n_nonneg=40, soc=(3, 4, 5, 6), psd=(2, 3, 5, 7),
                              n_exp=4, pow_alphas=tuple(rng.uniform(0.2, 0.8, 3)),
                              dpow_alphas=tuple(rng.uniform(0.2, 0.8, 3)))


def test_kkt_map_vanishes_at_the_known_solution(inst):
    q = inst
    g = D.G_map(q, q.x, q.y - q.s)
    assert np.linalg.norm(g) <= 1e-12 * (1 + np.linalg.norm(q.q) + np.linalg.norm(q.b))
    rng = np.random.default_rng(1)
    g2 = D.G_map(q, q.x + 1e-4 * rng.standard_normal(q.n), q.y - q.s)
    assert 1e-6 < np.linalg.norm(g2) < 1e-2


@pytest.mark.parametrize("eps", [1e-6, 1e-3])
def test_resolve_returns_to_the_known_solution(inst, eps):
    q = inst
    rng = np.random.default_rng(4)
    x0 = q.x + eps * rng.standard_normal(q.n)
    eta0 = q.y - q.s + eps * rng.standard_normal(q.m)
    x, y, s, res = D.newton_resolve(q, x0, eta0)
    assert res < 1e-13
    for a, b in zip((x, y, s), (q.x, q.y, q.s)):
        assert rel(a, b) < 1e-10
    # y in K*, s in K, complementary: y is its own projection onto K*, and by Moreau
    # Pi_{K*}(y - s) = y exactly when s = Pi_K(s) and y's = 0
    assert rel(C.proj_dual(y, q.cones), y) < 1e-12
    assert rel(C.proj_dual(y - s, q.cones), y) < 1e-12
    assert abs(y @ s) < 1e-12 * max(1.0, np.linalg.norm(y) * np.linalg.norm(s))
