"""Pins for the oracle's Jacobi scales (the column scaling of right-preconditioned LSQR).

The paper's least-squares solves (Sec. 3.1, 3.2) name no preconditioner; the reading taken
here is the diagonal (Jacobi) scaling D_jj = 1 / ||F_hat e_j||, where F_hat is the operator
F = (D_uQ - I) DPi + I of Sec. 2.4 with each cone block's Jacobian replaced by its diagonal.
The oracle computes those norms in closed form per kind of column and row. Here they are
checked against the norms of an explicitly assembled dense F_hat: D_uQ column by column from
the embedding's own product with D_uQ, the Jacobian diagonal probed one unit vector at a
time through the cone Jacobian's product. A planted mistake in the closed forms (a
column-dependent factor, the linear coefficient c written without its P x term, a dropped
b term) fails the pin.
"""
import numpy as np
import pytest

import qcpgen
from oracle import derivative as D
from oracle import embedding as E


def dense_F_hat(emb):
    N, n, m = emb.N, emb.n, emb.m
    DQ = np.empty((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        DQ[:, j] = emb.dq(e)
    jd = np.empty(m)
    for i in range(m):
        e = np.zeros(m)
        e[i] = 1.0
        jd[i] = emb.J.apply(e)[i]
    jhat = np.concatenate([np.ones(n), jd, [emb.dtau]])
    return (DQ - np.eye(N)) * jhat[None, :] + np.eye(N)


def scale_errors(emb, fcol=None, frow=None):
    Fh = dense_F_hat(emb)
    col = np.linalg.norm(Fh, axis=0)
    row = np.linalg.norm(Fh, axis=1)
    dcol = (fcol or D.jacobi_scale_F)(emb)
    drow = (frow or D.jacobi_scale_FT)(emb)
    return (np.max(np.abs(1.0 / dcol - col) / col), np.max(np.abs(1.0 / drow - row) / row))


CASES = {
    "tiny_qp": lambda: qcpgen.tiny_qp(0),
    "small_mixed": lambda: qcpgen.small_mixed(0),
    "medium_mixed": lambda: qcpgen.small_mixed(1, n=120, A_density=0.08, P_rank=30),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_jacobi_scales_are_dense_F_hat_norms(name):
    emb = E.Embedding(CASES[name]())
    ec, er = scale_errors(emb)
    assert ec <= 1e-13 and er <= 1e-13


def test_planted_column_factor_fails():
    emb = E.Embedding(qcpgen.small_mixed(0))
    f = np.linspace(0.3, 3.0, emb.N)
    ec, er = scale_errors(emb, fcol=lambda e: D.jacobi_scale_F(e) * f,
                          frow=lambda e: D.jacobi_scale_FT(e) * f)
    assert ec > 0.1 and er > 0.1


def test_planted_linear_coefficient_without_Px_fails():
    """c = -2 P x - q written as -q: the x columns of F and the tau row change."""
    emb = E.Embedding(qcpgen.small_mixed(0))
    Px = emb.Px.copy()

    def wrong(fn):
        def g(e):
            e.Px = np.zeros_like(Px)
            try:
                return fn(e)
            finally:
                e.Px = Px
        return g
    ec, er = scale_errors(emb, fcol=wrong(D.jacobi_scale_F), frow=wrong(D.jacobi_scale_FT))
    assert ec > 1e-3 and er > 1e-3


def test_planted_dropped_b_fails():
    """Dropping b (from the y columns of F and from the tau column and row): the scales of
    the y columns with a nonzero Jacobian diagonal and of the tau index change."""
    q = qcpgen.small_mixed(0)
    emb = E.Embedding(q)
    b = q.b.copy()

    def wrong(fn):
        def g(e):
            e.qcp.b = np.zeros_like(b)
            try:
                return fn(e)
            finally:
                e.qcp.b = b
        return g
    ec, er = scale_errors(emb, fcol=wrong(D.jacobi_scale_F), frow=wrong(D.jacobi_scale_FT))
    assert ec > 1e-3 and er > 1e-3
