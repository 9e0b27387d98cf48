"""Batched form: many QCPs of uneven sizes in one launch; each problem's outputs must match
the dense oracle (and the single-problem path) to the FP64 bar."""
import numpy as np
import pytest

import qcpgen
from oracle import derivative as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2508_17522_amd as Q  # noqa: E402
from qcpgen.torch_io import batch_create_args, batch_to_device  # noqa: E402

BAR = 1e-7


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def uneven_small(count=12):
    out = []
    rng = np.random.default_rng(77)
    for i in range(count):
        n = int(rng.integers(15, 90))
        nz = int(rng.integers(0, n // 4))
        nn = int(rng.integers(n // 4, n // 2))
        soc = tuple(int(k) for k in rng.integers(1, 7, size=int(rng.integers(0, 5))))
        psd = tuple(int(k) for k in rng.integers(1, 6, size=int(rng.integers(0, 3))))
        ne = int(rng.integers(0, 4))
        out.append(qcpgen.small_mixed(100 + i, n=n, n_zero=nz, n_nonneg=nn, soc=soc, psd=psd,
                                      n_exp=ne, A_density=0.15, P_rank=max(1, (3 * n) // 4),
                                      P_eps=0.05, nonneg_active=nn // 3))
    return out


def split(v, sizes):
    return np.split(v, np.cumsum(sizes)[:-1])


PRECONDS = [Q.QCPD_PRECOND_JACOBI, Q.QCPD_PRECOND_EQUIL]


@pytest.mark.parametrize("precond", PRECONDS)
def test_batch_matches_oracle_uneven(precond):
    qs = uneven_small()
    bt = batch_to_device(qs)
    h = Q.qcpd_batch_create(*batch_create_args(bt), opts=Q.Opts(tol=1e-12, precond=precond))
    dx, dy, ds, infos, st = Q.qcpd_batch_jvp(h, bt["dP"], bt["dA"], bt["dq"], bt["db"])
    print("jvp iters", [i.iters for i in infos], "status", st, flush=True)
    assert st == Q.QCPD_OK
    dxs = split(dx.cpu().numpy(), bt["n"])
    dys = split(dy.cpu().numpy(), bt["m"])
    dss = split(ds.cpu().numpy(), bt["m"])
    for k, q in enumerate(qs):
        ref = D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)
        errs = [rel(a, r) for a, r in zip((dxs[k], dys[k], dss[k]), ref)]
        assert max(errs) <= BAR, (k, errs)
        assert infos[k].rel_residual <= 1e-11
    dP, dA, dq, db, infos2, st2 = Q.qcpd_batch_vjp(h, bt["gx"], bt["gy"], bt["gs"])
    print("vjp iters", [i.iters for i in infos2], "status", st2, flush=True)
    assert st2 == Q.QCPD_OK
    dPs = split(dP.cpu().numpy(), bt["nnz_P"])
    dAs = split(dA.cpu().numpy(), bt["nnz_A"])
    dqs = split(dq.cpu().numpy(), bt["n"])
    dbs = split(db.cpu().numpy(), bt["m"])
    for k, q in enumerate(qs):
        ref = D.vjp_dense(q, q.gx, q.gy, q.gs)
        errs = [rel(a, r) for a, r in zip((dPs[k], dAs[k], dqs[k], dbs[k]), ref)]
        assert max(errs) <= BAR, (k, errs)
    h.close()


def test_batch_with_larger_psd_orders():
    """PSD cones of orders 20 and 40 in the batch (padded orders 32 and 48) run the batch's
    general F' kernel; the others have small cones only."""
    qs = [qcpgen.small_mixed(300, n=70, n_zero=5, n_nonneg=30, soc=(4, 3), psd=(20, 2),
                             n_exp=1, A_density=0.1, P_rank=60, P_eps=0.05, nonneg_active=10,
                             psd_ranks=(4, 1)),
          qcpgen.small_mixed(302, n=120, n_zero=5, n_nonneg=40, soc=(3,), psd=(40,), n_exp=2,
                             A_density=0.05, P_rank=100, P_eps=0.05, nonneg_active=15,
                             psd_ranks=(6,)),
          qcpgen.small_mixed(301, n=30, n_zero=3, n_nonneg=12, soc=(3,), psd=(3,), n_exp=0,
                             A_density=0.15, P_rank=25, P_eps=0.05, nonneg_active=4)]
    bt = batch_to_device(qs)
    h = Q.qcpd_batch_create(*batch_create_args(bt), opts=Q.Opts(tol=1e-12))
    dx, dy, ds, infos, st = Q.qcpd_batch_jvp(h, bt["dP"], bt["dA"], bt["dq"], bt["db"])
    print("jvp iters", [i.iters for i in infos], "status", st, flush=True)
    assert st == Q.QCPD_OK
    dxs, dys, dss = (split(v.cpu().numpy(), s) for v, s in
                     ((dx, bt["n"]), (dy, bt["m"]), (ds, bt["m"])))
    for k, q in enumerate(qs):
        ref = D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)
        errs = [rel(a, r) for a, r in zip((dxs[k], dys[k], dss[k]), ref)]
        assert max(errs) <= BAR, (k, errs)
    h.close()


@pytest.mark.parametrize("precond", PRECONDS)
def test_batch_of_one_matches_single_path(precond):
    q = qcpgen.small_mixed(0)
    bt = batch_to_device([q])
    h = Q.qcpd_batch_create(*batch_create_args(bt), opts=Q.Opts(tol=1e-12, precond=precond))
    dx, dy, ds, infos, st = Q.qcpd_batch_jvp(h, bt["dP"], bt["dA"], bt["dq"], bt["db"])
    from qcpgen.torch_io import cones_of, to_device
    t = to_device(q)
    hs = Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones_of(q), t["x"], t["y"], t["s"],
                       opts=Q.Opts(tol=1e-12, precond=precond))
    sx, sy, ss, info, st1 = Q.qcpd_jvp(hs, t["dP"], t["dA"], t["dq"], t["db"])
    for a, b in zip((dx, dy, ds), (sx, sy, ss)):
        assert rel(a.cpu().numpy(), b.cpu().numpy()) <= 1e-9


@pytest.mark.parametrize("precond", PRECONDS)
def test_batch_family_members_properties(precond):
    """Members of the uneven 20 <= n <= 400 family at the benchmark tolerance: the explicit
    relative residual of every problem and the adjoint identity per problem."""
    qs = [qcpgen.batch_member(i) for i in range(6)]
    bt = batch_to_device(qs)
    h = Q.qcpd_batch_create(*batch_create_args(bt), opts=Q.Opts(tol=1e-8, precond=precond))
    dx, dy, ds, i1, st = Q.qcpd_batch_jvp(h, bt["dP"], bt["dA"], bt["dq"], bt["db"])
    dP, dA, dq, db, i2, st2 = Q.qcpd_batch_vjp(h, bt["gx"], bt["gy"], bt["gs"])
    print("iters", [i.iters for i in i1], [i.iters for i in i2], st, st2, flush=True)
    assert st == Q.QCPD_OK and st2 == Q.QCPD_OK
    assert max(i.rel_residual for i in i1 + i2) <= 1e-8
    parts = [split(t.cpu().numpy(), s) for t, s in
             ((dx, bt["n"]), (dy, bt["m"]), (ds, bt["m"]), (dP, bt["nnz_P"]), (dA, bt["nnz_A"]),
              (dq, bt["n"]), (db, bt["m"]))]
    for k, q in enumerate(qs):
        lhs = q.gx @ parts[0][k] + q.gy @ parts[1][k] + q.gs @ parts[2][k]
        rhs = parts[3][k] @ q.dP + parts[4][k] @ q.dA + parts[5][k] @ q.dq + parts[6][k] @ q.db
        assert abs(lhs - rhs) <= 1e-4 * abs(lhs), (k, lhs, rhs)
