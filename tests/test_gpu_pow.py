"""Power and dual power cones (App. A) on the GPU: the operator F and the Jacobian diagonal at
points of every case of the appendix (interior of the cone or its polar, the plane z = 0 with
alpha below, at and above one half, the root-finding case), then JVP and VJP of programs with
power cones against the oracle's dense implicit-function solve (relative error <= 1e-7 at
tolerance 1e-12), the kink warning, and the batched form's refusal."""
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
from qcpgen.torch_io import batch_create_args, batch_to_device, cones_of, to_device  # noqa: E402

BAR = 1e-7


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def instance(idx=5, n=40, pw=(0.3, 0.5, 0.8), dp=(0.25, 0.6, 0.5), **kw):
    return qcpgen.small_mixed(idx, n=n, pow_alphas=pw, dpow_alphas=dp, P_eps=0.1, **kw)


def handle(q, tol=1e-12, precond=Q.QCPD_PRECOND_JACOBI):
    t = to_device(q)
    h = Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones_of(q), t["x"], t["y"], t["s"],
                      opts=Q.Opts(tol=tol, precond=precond))
    return h, t


def case_blocks(alphas):
    """(y, s) pairs per power block whose eta = y - s hits each case of the appendix for the
    projection the block's J evaluates (at -eta for a power cone, eta for a dual one)."""
    pts = []
    for a in alphas:
        x, y = 1.3, -0.4
        pts += [np.array([x, y, 0.0]), np.array([y, x, 0.0])]           # z = 0 case
        pts += [np.array([2.0, 1.5, 0.3]), np.array([-2.0, -1.5, 0.1])]  # interior / polar
        pts += [np.array([0.7, -1.2, 0.9]), np.array([-0.5, 0.4, -1.7])]  # root-finding
    return pts


@pytest.mark.parametrize("dual", [False, True])
def test_operator_and_jacobian_diagonal_in_every_case(dual):
    """Points not at a solution: the library's F, F' and diag J at z = (x, y - s, 1) against
    the oracle's (the product kernels apply whatever J the setup stored)."""
    alphas = (0.3, 0.5, 0.8)
    pts = case_blocks(alphas)
    per = len(pts) // len(alphas)
    al = [a for a in alphas for _ in range(per)]
    q = instance(idx=7, n=30, pw=() if dual else al, dp=al if dual else ())
    r0 = q.m - 3 * len(al)
    sg = 1.0 if dual else -1.0   # eta = y - s such that the evaluated point is the case point
    for i, pt in enumerate(pts):
        q.y[r0 + 3 * i:r0 + 3 * i + 3] = sg * pt
        q.s[r0 + 3 * i:r0 + 3 * i + 3] = 0.0
    h, t = handle(q)
    emb = E.Embedding(q)
    rng = np.random.default_rng(3)
    N = q.n + q.m + 1
    u, v = rng.standard_normal(N), rng.standard_normal(N)
    Fv = Q.qcpd_apply(h, torch.tensor(v, device="cuda")).cpu().numpy()
    FTu = Q.qcpd_apply(h, torch.tensor(u, device="cuda"), transpose=True).cpu().numpy()
    assert rel(Fv, emb.F(v)) <= 1e-12 and rel(FTu, emb.FT(u)) <= 1e-12
    jd = Q.qcpd_get_diagnostics(h)["jdiag"].cpu().numpy()
    ref = C.DualJacobian(q.y - q.s, q.cones).diagonal()
    assert np.abs(jd - ref).max() <= 1e-12
    h.close()


@pytest.mark.parametrize("case", ["small", "medium"])
def test_power_cone_program_matches_dense_oracle(case):
    if case == "small":
        q = instance()
    else:  # several 3 x 3 units, exponential and power cones side by side
        rng = np.random.default_rng(4)
        pw = tuple(float(a) for a in rng.uniform(0.1, 0.9, size=40))
        dp = tuple(float(a) for a in rng.uniform(0.1, 0.9, size=40)) + (0.5,) * 6
        q = instance(idx=8, n=301, n_zero=20, n_nonneg=200, soc=(3, 5) * 5, psd=(4, 6),
                     n_exp=30, pw=pw, dp=dp, A_density=0.04, P_rank=150, nonneg_active=60)
    for precond in (Q.QCPD_PRECOND_JACOBI, Q.QCPD_PRECOND_EQUIL):
        h, t = handle(q, precond=precond)
        assert h.create_status == Q.QCPD_OK
        dx, dy, ds, info, st = Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"])
        print(f"[{case} {precond}] jvp iters={info.iters} rel={info.rel_residual:.2e} st={st}",
              flush=True)
        assert st == Q.QCPD_OK
        ref = D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)
        errs = [rel(a.cpu().numpy(), b) for a, b in zip((dx, dy, ds), ref)]
        print(f"[{case}] jvp errors {errs}", flush=True)
        assert max(errs) <= BAR
        dP, dA, dq, db, info2, st2 = Q.qcpd_vjp(h, t["gx"], t["gy"], t["gs"])
        assert st2 == Q.QCPD_OK
        refv = D.vjp_dense(q, q.gx, q.gy, q.gs)
        errs2 = [rel(a.cpu().numpy(), b) for a, b in zip((dP, dA, dq, db), refv)]
        print(f"[{case}] vjp errors {errs2}", flush=True)
        assert max(errs2) <= BAR
        h.close()


def test_power_cone_on_its_boundary_is_reported():
    """A power block whose evaluated point lies on the cone's boundary: a kink."""
    q = instance(idx=9, n=30, pw=(0.4,), dp=())
    r0 = q.m - 3
    x, y = 1.2, 0.7
    q.y[r0:r0 + 3] = -np.array([x, y, x ** 0.4 * y ** 0.6])   # -eta on the boundary of K
    q.s[r0:r0 + 3] = 0.0
    t = to_device(q)
    h = Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones_of(q), t["x"], t["y"], t["s"])
    assert h.create_status == Q.QCPD_WARN_NONDIFF
    h.close()


def test_bad_exponent_and_batch_are_refused():
    q = instance(idx=10, n=30, pw=(0.4,), dp=())
    t = to_device(q)
    bad = cones_of(q)
    bad.pow = [1.0]
    with pytest.raises(Q.QCPDError) as e:
        Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], bad, t["x"], t["y"], t["s"])
    assert e.value.status == Q.QCPD_ERR_CONE
    bt = batch_to_device([q])
    with pytest.raises(Q.QCPDError) as e:
        Q.qcpd_batch_create(*batch_create_args(bt))
    assert e.value.status == Q.QCPD_ERR_CONE
