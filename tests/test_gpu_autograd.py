"""torch.autograd integration: backward is the library's VJP, forward-mode is its JVP.

Checked against the dense oracle and against central finite differences (step 1e-6) of
loss = ||x*(theta) - x_target||^2 through a Newton re-solve of the perturbed problems, on a
member of the uneven batched family (n in [20, 400])."""
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
from qcpgen.torch_io import cones_of, to_device  # noqa: E402


def structure(qcp, t, tol=1e-12, max_iter=0):
    return Q.QCPStructure(t["P"][0], t["P"][1], t["A"][0], t["A"][1], cones_of(qcp),
                          Q.Opts(tol=tol, max_iter=max_iter))


def leaves(t):
    return [t["P"][2].clone().requires_grad_(), t["A"][2].clone().requires_grad_(),
            t["q"].clone().requires_grad_(), t["b"].clone().requires_grad_()]


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_backward_matches_oracle_vjp():
    q = qcpgen.small_mixed(0)
    t = to_device(q)
    P, A, qq, b = leaves(t)
    x, y, s = Q.qcp_solution_map(P, A, qq, b, t["x"], t["y"], t["s"], structure(q, t))
    loss = (x * t["gx"]).sum() + (y * t["gy"]).sum() + (s * t["gs"]).sum()
    loss.backward()
    ref = D.vjp_dense(q, q.gx, q.gy, q.gs)
    for g, r in zip((P.grad, A.grad, qq.grad, b.grad), ref):
        assert rel(g.cpu().numpy(), r) < 1e-7


def test_forward_mode_matches_oracle_jvp():
    import torch.autograd.forward_ad as fwAD
    q = qcpgen.small_mixed(0)
    t = to_device(q)
    st = structure(q, t)
    with fwAD.dual_level():
        P = fwAD.make_dual(t["P"][2], t["dP"])
        A = fwAD.make_dual(t["A"][2], t["dA"])
        qq = fwAD.make_dual(t["q"], t["dq"])
        b = fwAD.make_dual(t["b"], t["db"])
        out = Q.qcp_solution_map(P, A, qq, b, t["x"], t["y"], t["s"], st)
        tang = [fwAD.unpack_dual(o).tangent for o in out]
    ref = D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)
    for a, r in zip(tang, ref):
        assert rel(a.cpu().numpy(), r) < 1e-7


def test_loss_gradient_against_finite_differences():
    q = qcpgen.batch_member(2)
    rng = np.random.default_rng(123)
    x_target = rng.standard_normal(q.n)
    t = to_device(q)
    P, A, qq, b = leaves(t)
    x, y, s = Q.qcp_solution_map(P, A, qq, b, t["x"], t["y"], t["s"],
                                 structure(q, t, max_iter=1_000_000))
    xt = torch.as_tensor(x_target, device=x.device)
    loss = ((x - xt) ** 2).sum()
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("error")  # a non-converged LSQR fails the test
        loss.backward()
    # directional derivative along the generator's perturbation (dP symmetric on pattern)
    got = (P.grad.cpu().numpy() @ q.dP + A.grad.cpu().numpy() @ q.dA
           + qq.grad.cpu().numpy() @ q.dq + b.grad.cpu().numpy() @ q.db)
    h = 1e-6
    vals = []
    for sgn in (+1, -1):
        qh = E.with_data(q, q.dP, q.dA, q.dq, q.db, h=sgn * h)
        xs, ys, ss, res = D.newton_resolve(qh, q.x, q.y - q.s)
        assert res < 1e-12
        vals.append(np.sum((xs - x_target) ** 2))
    fd = (vals[0] - vals[1]) / (2 * h)
    print(f"n={q.n} m={q.m} grad.dtheta={got:.12e} fd={fd:.12e}", flush=True)
    assert abs(got - fd) <= 1e-6 * max(abs(fd), 1e-3)
