"""Batched torch.autograd: many problems of the uneven 20 <= n <= 400 family in one batch
handle, loss = sum over problems of ||x*(theta) - x_target||^2, gradients by one batched VJP.
Checked per problem against the oracle's dense adjoint and against central differences
(step 1e-6) of the loss through a Newton re-solve of the perturbed problems; forward mode
against the dense derivative."""
import numpy as np
import pytest

import qcpgen
from oracle import derivative as D
from oracle import embedding as E

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2508_17522_amd as Q  # noqa: E402
from qcpgen.torch_io import batch_to_device  # noqa: E402

COUNT = 12


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def split(v, sizes):
    return np.split(np.asarray(v), np.cumsum(sizes)[:-1])


@pytest.fixture(scope="module")
def family():
    qs = [qcpgen.batch_member(i) for i in range(COUNT)]
    bt = batch_to_device(qs)
    st = Q.BatchStructure(bt["n"], bt["m"], bt["nnz_P"], bt["nnz_A"], bt["cones"],
                          bt["P_rowptr"], bt["P_colind"], bt["A_rowptr"], bt["A_colind"],
                          Q.Opts(tol=1e-12, precond=Q.QCPD_PRECOND_EQUIL))
    rng = np.random.default_rng(2024)
    xt = rng.standard_normal(sum(bt["n"]))
    return qs, bt, st, xt


def loss_and_grads(bt, st, xt):
    P = bt["P_val"].clone().requires_grad_()
    A = bt["A_val"].clone().requires_grad_()
    qq = bt["q"].clone().requires_grad_()
    b = bt["b"].clone().requires_grad_()
    x, y, s = Q.batch_solution_map(P, A, qq, b, bt["x"], bt["y"], bt["s"], st)
    target = torch.tensor(xt, device=x.device)
    loss = ((x - target) ** 2).sum()
    loss.backward()
    return loss.item(), [g.detach().cpu().numpy() for g in (P.grad, A.grad, qq.grad, b.grad)]


def test_batched_backward_matches_dense_adjoint(family):
    qs, bt, st, xt = family
    _, grads = loss_and_grads(bt, st, xt)
    parts = [split(g, s) for g, s in zip(grads, (bt["nnz_P"], bt["nnz_A"], bt["n"], bt["m"]))]
    xts = split(xt, bt["n"])
    for k, q in enumerate(qs):
        gx = 2.0 * (q.x - xts[k])
        ref = D.vjp_dense(q, gx, np.zeros(q.m), np.zeros(q.m))
        errs = [rel(p[k], r) for p, r in zip(parts, ref)]
        assert max(errs) <= 1e-7, (k, errs)


def test_batched_gradient_against_finite_differences(family):
    """d loss / d theta along random directions, for several members: <grad, dtheta> (pattern
    inner products) against central differences of the loss with each perturbed problem
    re-solved by Newton's method."""
    qs, bt, st, xt = family
    _, grads = loss_and_grads(bt, st, xt)
    parts = [split(g, s) for g, s in zip(grads, (bt["nnz_P"], bt["nnz_A"], bt["n"], bt["m"]))]
    xts = split(xt, bt["n"])
    h = 1e-6
    rng = np.random.default_rng(7)
    worst = 0.0
    for k in (0, 3, 7):
        q = qs[k]
        for _ in range(2):
            dP = qcpgen.symmetric_on_pattern(rng, q.P, 1.0)
            dA = rng.standard_normal(q.A.nnz)
            dq = rng.standard_normal(q.n)
            db = rng.standard_normal(q.m)
            ana = (parts[0][k] @ dP + parts[1][k] @ dA + parts[2][k] @ dq + parts[3][k] @ db)
            vals = []
            for sgn in (1.0, -1.0):
                qp = E.with_data(q, dP, dA, dq, db, h=sgn * h)
                xp, _, _, res = D.newton_resolve(qp, q.x, q.y - q.s)
                assert res < 1e-13
                vals.append(float(((xp - xts[k]) ** 2).sum()))
            fd = (vals[0] - vals[1]) / (2 * h)
            err = abs(fd - ana) / max(abs(ana), 1e-12)
            worst = max(worst, err)
            assert err <= 1e-5, (k, fd, ana)  # truncation of the step-1e-6 differences: ~1e-6
    print(f"worst relative difference, gradient vs differences: {worst:.2e}", flush=True)


def test_batched_forward_mode_matches_dense(family):
    import torch.autograd.forward_ad as fwAD
    qs, bt, st, xt = family
    with fwAD.dual_level():
        P = fwAD.make_dual(bt["P_val"], bt["dP"])
        A = fwAD.make_dual(bt["A_val"], bt["dA"])
        qq = fwAD.make_dual(bt["q"], bt["dq"])
        b = fwAD.make_dual(bt["b"], bt["db"])
        out = Q.batch_solution_map(P, A, qq, b, bt["x"], bt["y"], bt["s"], st)
        tang = [fwAD.unpack_dual(o).tangent.cpu().numpy() for o in out]
    parts = [split(v, s) for v, s in zip(tang, (bt["n"], bt["m"], bt["m"]))]
    for k, q in enumerate(qs):
        ref = D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)
        assert max(rel(p[k], r) for p, r in zip(parts, ref)) <= 1e-7, k
