"""The forward solve by refinement (qcpd_resolve) and the projection onto K* it rests on
(qcpd_proj_dual), against the oracle: Pi_{K*} of random points for every cone type
(nonnegative, SOC, PSD, exponential, power, dual power) within 1e-11; Newton's method from
the old solution after a step in theta against the oracle's dense semismooth Newton
re-solve of the same perturbed instance (1e-9), and from a perturbed point of an unchanged
instance back to its known solution (1e-9)."""
import numpy as np
import pytest

import qcpgen
from oracle import cones as C
from oracle import derivative as D
from oracle import embedding as E

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2508_17522_amd as Q  # noqa: E402
from qcpgen.torch_io import cones_of, to_device  # noqa: E402


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1.0)


def instance(idx=0):
    rng = np.random.default_rng([31, idx])
    return qcpgen.small_mixed(idx, n=60, n_zero=6, n_nonneg=40, soc=(3, 4, 5, 6),
                              psd=(2, 3, 5, 7), n_exp=4, pow_alphas=tuple(rng.uniform(0.2, 0.8, 3)),
                              dpow_alphas=tuple(rng.uniform(0.2, 0.8, 3)))


def handle(q):
    t = to_device(q)
    h = Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones_of(q), t["x"], t["y"], t["s"])
    return h, t


@pytest.mark.parametrize("scale", [0.3, 1.0, 5.0])
def test_proj_dual_matches_oracle(scale):
    q = instance(0)
    h, t = handle(q)
    rng = np.random.default_rng(5)
    for trial in range(3):
        zy = scale * rng.standard_normal(q.m)
        out = Q.qcpd_proj_dual(h, torch.tensor(zy, device="cuda:0")).cpu().numpy()
        ref = C.proj_dual(zy, q.cones)
        err = np.abs(out - ref).max() / max(1.0, np.abs(zy).max())
        print(f"scale {scale} trial {trial}: max error {err:.2e}", flush=True)
        assert err <= 1e-11
    # at the solution, Pi_{K*}(y - s) = y
    out = Q.qcpd_proj_dual(h, t["y"] - t["s"]).cpu().numpy()
    assert np.abs(out - q.y).max() <= 1e-12 * max(1.0, np.abs(q.y).max())
    h.close()


def test_resolve_after_a_step_in_theta_matches_oracle_newton():
    q = instance(1)
    rng = np.random.default_rng(9)
    dP = qcpgen.symmetric_on_pattern(rng, q.P, 1.0)
    dA, dq, db = rng.standard_normal(q.A.nnz), rng.standard_normal(q.n), rng.standard_normal(q.m)
    qp = E.with_data(q, dP, dA, dq, db, h=1e-3)
    xr, yr, sr, res = D.newton_resolve(qp, q.x, q.y - q.s)
    assert res < 1e-13
    t = to_device(qp)
    t0 = to_device(q)
    x, y, s, info, st = Q.qcpd_resolve(t["P"], t["A"], t["q"], t["b"], cones_of(qp), t0["x"],
                                       t0["y"], t0["s"], tol=1e-12,
                                       opts=Q.Opts(tol=1e-12, precond=Q.QCPD_PRECOND_EQUIL))
    print(f"newton {info.newton_iters} lsqr {info.lsqr_iters} residual {info.residual:.2e} st {st}",
          flush=True)
    assert st == Q.QCPD_OK and info.converged and info.newton_iters >= 1
    errs = [rel(a.cpu().numpy(), b) for a, b in zip((x, y, s), (xr, yr, sr))]
    print(f"x y s against the oracle: {['%.1e' % e for e in errs]}", flush=True)
    assert max(errs) <= 1e-9
    # the returned point is a solution: primal and dual feasibility, complementarity
    xn, yn, sn = (v.cpu().numpy() for v in (x, y, s))
    g = D.G_map(qp, xn, yn - sn)
    assert np.linalg.norm(g) <= 1e-11 * (1 + np.linalg.norm(qp.q) + np.linalg.norm(qp.b))
    assert abs(yn @ sn) <= 1e-11 * max(1.0, np.linalg.norm(yn) * np.linalg.norm(sn))


def test_resolve_returns_to_the_known_solution():
    q = instance(2)
    rng = np.random.default_rng(4)
    t = to_device(q)
    x0 = t["x"] + 1e-3 * torch.tensor(rng.standard_normal(q.n), device="cuda:0")
    y0 = t["y"] + 1e-3 * torch.tensor(rng.standard_normal(q.m), device="cuda:0")
    x, y, s, info, st = Q.qcpd_resolve(t["P"], t["A"], t["q"], t["b"], cones_of(q), x0, y0,
                                       t["s"], tol=1e-12, opts=Q.Opts(tol=1e-12))
    print(f"newton {info.newton_iters} residual {info.residual:.2e}", flush=True)
    assert st == Q.QCPD_OK and info.converged
    errs = [rel(a.cpu().numpy(), b) for a, b in zip((x, y, s), (q.x, q.y, q.s))]
    print(f"x y s against the known solution: {['%.1e' % e for e in errs]}", flush=True)
    assert max(errs) <= 1e-9


def test_resolve_at_a_solution_takes_no_step_and_rejects_bad_arguments():
    q = instance(0)
    t = to_device(q)
    x, y, s, info, st = Q.qcpd_resolve(t["P"], t["A"], t["q"], t["b"], cones_of(q), t["x"],
                                       t["y"], t["s"], tol=1e-10)
    assert st == Q.QCPD_OK and info.newton_iters == 0 and info.residual <= 1e-10
    x0 = t["x"] + 1e-2
    _, _, _, info, st = Q.qcpd_resolve(t["P"], t["A"], t["q"], t["b"], cones_of(q), x0, t["y"],
                                       t["s"], tol=1e-12, max_newton=0)
    assert st == Q.QCPD_WARN_NOT_CONVERGED and not info.converged and info.residual > 1e-12
    with pytest.raises(Q.QCPDError) as e:
        Q.qcpd_resolve(t["P"], t["A"], t["q"], t["b"], cones_of(q), t["x"], t["y"], t["s"],
                       tol=0.0)
    assert e.value.status == Q.QCPD_ERR_INVALID_ARG


def test_learning_loop_refines_and_differentiates():
    """A small synthetic learning loop (Sec. 3.4 without its comparison systems): theta =
    (q, b) moves by gradient steps on ||x*(theta) - x_target||^2; each forward refines the
    previous solution to the current data (QCPStructure.refine_tol) and each backward is the
    library's adjoint. Per step: the refined solution against the oracle's re-solve of the
    same data from the same start (1e-9), the gradients against the oracle's dense adjoint at
    that solution (1e-7); the loss decreases."""
    q0 = instance(3)
    t0 = to_device(q0)
    st = Q.QCPStructure(t0["P"][0], t0["P"][1], t0["A"][0], t0["A"][1], cones_of(q0),
                        Q.Opts(tol=1e-12, precond=Q.QCPD_PRECOND_EQUIL), refine_tol=1e-12)
    rng = np.random.default_rng(12)
    xt = q0.x + 0.1 * rng.standard_normal(q0.n)
    xt_d = torch.tensor(xt, device="cuda:0")
    qv, bv = t0["q"].clone(), t0["b"].clone()
    x, y, s = t0["x"], t0["y"], t0["s"]
    losses = []
    for k in range(4):
        qp = qv.clone().requires_grad_()
        bp = bv.clone().requires_grad_()
        xs, ys, ss = Q.qcp_solution_map(t0["P"][2], t0["A"][2], qp, bp, x, y, s, st)
        loss = ((xs - xt_d) ** 2).sum()
        loss.backward()
        qk = E.with_data(q0, dq=qv.cpu().numpy() - q0.q, db=bv.cpu().numpy() - q0.b)
        xr, yr, sr, res = D.newton_resolve(qk, x.cpu().numpy(), (y - s).cpu().numpy())
        assert res < 1e-12
        errs = [rel(a.detach().cpu().numpy(), b) for a, b in zip((xs, ys, ss), (xr, yr, sr))]
        qk.x, qk.y, qk.s = xr, yr, sr
        ref = D.vjp_dense(qk, 2.0 * (xr - xt), np.zeros(q0.m), np.zeros(q0.m))
        gerr = max(rel(qp.grad.cpu().numpy(), ref[2]), rel(bp.grad.cpu().numpy(), ref[3]))
        print(f"step {k}: loss {loss.item():.6e} solution {['%.1e' % e for e in errs]} "
              f"gradient {gerr:.1e}", flush=True)
        assert max(errs) <= 1e-9 and gerr <= 1e-7
        losses.append(loss.item())
        with torch.no_grad():  # steps of 1e-3 relative in theta keep each refinement local
            g = torch.cat([qp.grad, bp.grad])
            lr = 1e-3 * torch.cat([qv, bv]).norm() / g.norm()
            qv -= lr * qp.grad
            bv -= lr * bp.grad
        x, y, s = xs.detach(), ys.detach(), ss.detach()
    assert losses[-1] < losses[0]
