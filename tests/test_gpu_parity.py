"""GPU parity: the HIP library (through its C-ABI) against the CPU oracle.

Bar (FP64): relative 2-norm error <= 1e-7 on dx, dy, ds and on dP, dA, dq, db. The least
squares problems are solved to a relative residual of 1e-12 here so that the forward error,
which can reach cond(K_red) x tol, stays well below the bar; the oracle reference is the
dense implicit-function solve (exact up to rounding) where it is affordable.
"""
import math

import numpy as np
import pytest

import qcpgen
from oracle import derivative as D
from oracle import embedding as E

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU machines, skipped there
    pytest.skip("no GPU", allow_module_level=True)

import paper_2508_17522_amd as Q  # noqa: E402
from qcpgen.torch_io import cones_of, to_device  # noqa: E402

BAR = 1e-7


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def make_handle(qcp, tol=1e-12, precond=Q.QCPD_PRECOND_JACOBI, max_iter=0, chunk=32,
                engine=Q.QCPD_ENGINE_AUTO, **layout):
    t = to_device(qcp)
    o = Q.Opts(tol=tol, max_iter=max_iter, precond=precond, graph_chunk=chunk, engine=engine,
               **layout)
    h = Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones_of(qcp), t["x"], t["y"], t["s"], opts=o)
    return h, t


def gpu_jvp(h, t):
    dx, dy, ds, info, st = Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"])
    return dx.cpu().numpy(), dy.cpu().numpy(), ds.cpu().numpy(), info, st


def gpu_vjp(h, t):
    dP, dA, dq, db, info, st = Q.qcpd_vjp(h, t["gx"], t["gy"], t["gs"])
    return dP.cpu().numpy(), dA.cpu().numpy(), dq.cpu().numpy(), db.cpu().numpy(), info, st


def check_jvp_vjp_dense(qcp, tol=1e-12, **kw):
    h, t = make_handle(qcp, tol=tol, **kw)
    dx, dy, ds, info, st = gpu_jvp(h, t)
    print(f"[{qcp.name}] jvp iters={info.iters} rel_res={info.rel_residual:.2e} st={st}", flush=True)
    assert st == Q.QCPD_OK
    assert info.rel_residual <= 10 * tol
    ref = D.jvp_dense(qcp, qcp.dP, qcp.dA, qcp.dq, qcp.db)
    errs = [rel(a, b) for a, b in zip((dx, dy, ds), ref)]
    print(f"[{qcp.name}] jvp errors {errs}", flush=True)
    assert max(errs) <= BAR
    dP, dA, dq, db, info2, st2 = gpu_vjp(h, t)
    print(f"[{qcp.name}] vjp iters={info2.iters} rel_res={info2.rel_residual:.2e} st={st2}", flush=True)
    assert st2 == Q.QCPD_OK
    refv = D.vjp_dense(qcp, qcp.gx, qcp.gy, qcp.gs)
    errs2 = [rel(a, b) for a, b in zip((dP, dA, dq, db), refv)]
    print(f"[{qcp.name}] vjp errors {errs2}", flush=True)
    assert max(errs2) <= BAR
    h.close()


# ---- small instances, dense oracle ----------------------------------------------------

@pytest.mark.parametrize("idx", [0, 1])
def test_tiny_qp(idx):
    check_jvp_vjp_dense(qcpgen.tiny_qp(idx))


def test_small_mixed_all_cones():
    check_jvp_vjp_dense(qcpgen.small_mixed(0))


@pytest.mark.parametrize("engine", [Q.QCPD_ENGINE_GRAPH, Q.QCPD_ENGINE_PERSISTENT])
def test_medium_mixed_several_tiles(engine):
    """Every cone type, several workgroups per region and ragged tails (n, m not multiples
    of the tile), PSD orders up to 12; both LSQR drivers."""
    q = qcpgen.small_mixed(1, n=301, n_zero=37, n_nonneg=260, soc=(3, 4, 5, 6, 7, 8) * 5,
                           psd=(4, 7, 12, 9), n_exp=23, A_density=0.04, P_rank=150,
                           nonneg_active=100)
    check_jvp_vjp_dense(q, engine=engine)


@pytest.mark.parametrize("precond", [Q.QCPD_PRECOND_NONE, Q.QCPD_PRECOND_EQUIL])
def test_other_preconditioners_match(precond):
    q = qcpgen.small_mixed(0)
    check_jvp_vjp_dense(q, precond=precond)


def test_equilibrated_medium_and_custom_scaling():
    """Two-sided equilibration on every cone type, then the same scales passed back in as a
    custom two-sided preconditioner."""
    q = qcpgen.small_mixed(1, n=301, n_zero=37, n_nonneg=260, soc=(3, 4, 5, 6, 7, 8) * 5,
                           psd=(4, 7, 12, 9), n_exp=23, A_density=0.04, P_rank=150,
                           nonneg_active=100)
    check_jvp_vjp_dense(q, precond=Q.QCPD_PRECOND_EQUIL)
    h, t = make_handle(q, precond=Q.QCPD_PRECOND_CUSTOM)
    dg = Q.qcpd_get_diagnostics(h)
    assert torch.all(dg["equil_col"] > 0) and torch.all(dg["equil_row"] > 0)
    Q.qcpd_set_precond(h, dg["equil_col"], dg["equil_row"])
    dx, dy, ds, info, st = gpu_jvp(h, t)
    ref = D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)
    assert st == Q.QCPD_OK and max(rel(a, b) for a, b in zip((dx, dy, ds), ref)) <= BAR


def test_psd_max_order():
    """A 64 x 64 PSD block (the largest order held in LDS) next to a 1 x 1 block."""
    q = qcpgen.small_mixed(2, n=200, n_zero=10, n_nonneg=40, soc=(1, 2), psd=(64, 1), n_exp=2,
                           A_density=0.02, P_rank=150, P_eps=1e-2, nonneg_active=15,
                           psd_ranks=(12, 1))
    check_jvp_vjp_dense(q)


@pytest.mark.parametrize("precond", [Q.QCPD_PRECOND_JACOBI, Q.QCPD_PRECOND_EQUIL])
def test_deep_csr_form_matches_oracle(precond):
    """The F' loop kernel's deep-CSR form (chosen by the library for large problems) forced
    on a small one with every cone type, in its single-unit and looping launch shapes."""
    q = qcpgen.small_mixed(1)
    layout = dict(deep=Q.QCPD_CHOICE_ON, staged=Q.QCPD_CHOICE_OFF)
    check_jvp_vjp_dense(q, precond=precond, **layout)
    h, t = make_handle(q, precond=precond, **layout)
    gF, gT, mF, mT = Q.qcpd_get_launch(h)
    Q.qcpd_set_launch(h, gF, max(1, mT // 3))  # fewer workgroups than units: looping form
    dx, dy, ds, info, st = gpu_jvp(h, t)
    assert st == Q.QCPD_OK
    ref = D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)
    errs = [rel(a, b) for a, b in zip((dx, dy, ds), ref)]
    print(f"deep, looping form: iters={info.iters} errors {errs}", flush=True)
    assert max(errs) <= BAR
    h.close()


@pytest.mark.parametrize("deep", [Q.QCPD_CHOICE_OFF, Q.QCPD_CHOICE_ON])
def test_psd_cones_in_their_own_launch(deep):
    """PSD cones of order above 32 run in a launch of their own after the rows launch of the
    product with F' (their raw rows pass through a buffer): plain and deep CSR sums, the
    single-unit and the looping launch shapes, every other cone type beside them."""
    q = qcpgen.small_mixed(4, n=150, n_zero=10, n_nonneg=60, soc=(3, 4, 5) * 3, psd=(40, 6, 33),
                           n_exp=5, A_density=0.03, P_rank=120, P_eps=1e-2, nonneg_active=20,
                           psd_ranks=(8, 2, 5))
    layout = dict(deep=deep, staged=Q.QCPD_CHOICE_OFF)
    check_jvp_vjp_dense(q, precond=Q.QCPD_PRECOND_EQUIL, **layout)
    h, t = make_handle(q, precond=Q.QCPD_PRECOND_EQUIL, **layout)
    gF, gT, mF, mT = Q.qcpd_get_launch(h)
    Q.qcpd_set_launch(h, gF, max(1, mT // 3))  # fewer workgroups than units: looping form
    dx, dy, ds, info, st = gpu_jvp(h, t)
    assert st == Q.QCPD_OK
    ref = D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)
    errs = [rel(a, b) for a, b in zip((dx, dy, ds), ref)]
    print(f"split, looping form: iters={info.iters} errors {errs}", flush=True)
    assert max(errs) <= BAR
    h.close()


def test_only_zero_cone_and_graph_chunk_one():
    q = qcpgen.small_mixed(3, n=30, n_zero=12, n_nonneg=0, soc=(), psd=(), n_exp=0,
                           A_density=0.3, P_rank=25, P_eps=0.1)
    check_jvp_vjp_dense(q, chunk=1)


# ---- the 5000 x 11000 mixed-cone workload at full size ----------------------------------

def kkt_linearised_residual(qcp, dx, dy, ds):
    """Residuals of the linearised optimality conditions that (dx, dy, ds) must satisfy:
    P dx + dP x + A'dy + dA'y + dq = 0,  A dx + dA x + ds - db = 0,  dy = J (dy - ds)."""
    from oracle import cones as C
    dPm = qcp.P.copy(); dPm.data = qcp.dP.copy()
    dAm = qcp.A.copy(); dAm.data = qcp.dA.copy()
    r1 = qcp.P @ dx + dPm @ qcp.x + qcp.A.T @ dy + dAm.T @ qcp.y + qcp.dq
    r2 = qcp.A @ dx + dAm @ qcp.x + ds - qcp.db
    J = C.DualJacobian(qcp.y - qcp.s, qcp.cones)
    r3 = dy - J.apply(dy - ds)
    scale = (np.linalg.norm(dPm @ qcp.x) + np.linalg.norm(dAm.T @ qcp.y) + np.linalg.norm(qcp.dq)
             + np.linalg.norm(dAm @ qcp.x) + np.linalg.norm(qcp.db))
    return (np.linalg.norm(r1) + np.linalg.norm(r2) + np.linalg.norm(r3)) / scale


@pytest.fixture(scope="module")
def mixed_full():
    return qcpgen.mixed_qcp(0)


@pytest.mark.parametrize("engine,precond", [(Q.QCPD_ENGINE_GRAPH, Q.QCPD_PRECOND_EQUIL),
                                            (Q.QCPD_ENGINE_GRAPH, Q.QCPD_PRECOND_JACOBI),
                                            (Q.QCPD_ENGINE_PERSISTENT, Q.QCPD_PRECOND_EQUIL)])
def test_mixed_full_size_properties(mixed_full, engine, precond):
    """At the benchmark size and tolerance: the JVP satisfies the linearised KKT system
    (oracle J and data, any size) and JVP/VJP satisfy the adjoint identity."""
    check_full_size(mixed_full, engine, precond, "mixed full")


def check_full_size(q, engine, precond, tag):
    h, t = make_handle(q, tol=1e-8, engine=engine, precond=precond)
    dx, dy, ds, info, st = gpu_jvp(h, t)
    print(f"[{tag}] jvp iters={info.iters} rel_res={info.rel_residual:.2e} "
          f"ms={info.ms_total:.1f} st={st}", flush=True)
    assert st == Q.QCPD_OK and info.rel_residual <= 1e-8
    res = kkt_linearised_residual(q, dx, dy, ds)
    print(f"[{tag}] linearised KKT residual {res:.2e}", flush=True)
    assert res <= 1e-6
    dP, dA, dq, db, info2, st2 = gpu_vjp(h, t)
    print(f"[{tag}] vjp iters={info2.iters} rel_res={info2.rel_residual:.2e} "
          f"ms={info2.ms_total:.1f} st={st2}", flush=True)
    assert st2 == Q.QCPD_OK and info2.rel_residual <= 1e-8
    lhs = q.gx @ dx + q.gy @ dy + q.gs @ ds
    rhs = dP @ q.dP + dA @ q.dA + dq @ q.dq + db @ q.db
    print(f"[{tag}] adjoint identity {lhs:.10e} {rhs:.10e}", flush=True)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    h.close()


def check_operator(q, h, seed=3, bar=1e-12):
    """F v and F'v of the library against the oracle's operator, on random v."""
    emb = E.Embedding(q)
    rng = np.random.default_rng(seed)
    N = q.n + q.m + 1
    u, v = rng.standard_normal(N), rng.standard_normal(N)
    Fv = Q.qcpd_apply(h, torch.tensor(v, device="cuda")).cpu().numpy()
    FTu = Q.qcpd_apply(h, torch.tensor(u, device="cuda"), transpose=True).cpu().numpy()
    e1, e2 = rel(Fv, emb.F(v)), rel(FTu, emb.FT(u))
    print(f"[{q.name}] operator errors F {e1:.1e} F' {e2:.1e}; <u,Fv> - <F'u,v> = "
          f"{abs(u @ Fv - FTu @ v) / (np.linalg.norm(u) * np.linalg.norm(Fv)):.1e}", flush=True)
    assert e1 <= bar and e2 <= bar
    assert abs(u @ Fv - FTu @ v) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(Fv)


def test_operator_matches_oracle_small_and_mixed(mixed_full):
    for q in (qcpgen.small_mixed(0), qcpgen.small_mixed(1, n=301, n_zero=37, n_nonneg=260,
                                                        soc=(3, 4, 5, 6, 7, 8) * 5,
                                                        psd=(4, 7, 12, 9), n_exp=23,
                                                        A_density=0.04, P_rank=150,
                                                        nonneg_active=100), mixed_full):
        h, t = make_handle(q, tol=1e-8)
        check_operator(q, h)
        h.close()


def test_large_psd_soc_full_size():
    """n = 20 000, m = 290 000 (200 PSD cones of order 50, 2 000 SOC(10)) at the benchmark
    tolerance: the operator against the oracle's, both directions converged (explicit
    residual <= 1e-8), the JVP satisfies the linearised KKT system, and JVP and VJP satisfy
    the adjoint identity. A reduced instance of the same shape is compared with the dense
    oracle entry by entry in test_gpu_fullsize.py."""
    q = qcpgen.large_psd_soc(0)
    print(f"[large] n={q.n} m={q.m} nnz P={q.P.nnz} nnz A={q.A.nnz}", flush=True)
    h, t = make_handle(q, tol=1e-8, precond=Q.QCPD_PRECOND_EQUIL)
    check_operator(q, h)
    h.close()
    check_full_size(q, Q.QCPD_ENGINE_GRAPH, Q.QCPD_PRECOND_EQUIL, "large")


# ---- edge cases and errors ----------------------------------------------------------------

def test_zero_perturbation_and_zero_cotangent():
    q = qcpgen.small_mixed(0)
    h, t = make_handle(q)
    for k in ("dP", "dA", "dq", "db", "gx", "gy", "gs"):
        t[k] = torch.zeros_like(t[k])
    dx, dy, ds, info, st = gpu_jvp(h, t)
    assert st == Q.QCPD_OK and info.iters == 0
    assert not np.any(dx) and not np.any(dy) and not np.any(ds)
    dP, dA, dq, db, info, st = gpu_vjp(h, t)
    assert st == Q.QCPD_OK and not np.any(dP) and not np.any(dq)


@pytest.mark.parametrize("engine", [Q.QCPD_ENGINE_GRAPH, Q.QCPD_ENGINE_PERSISTENT])
def test_not_converged_warning(engine):
    q = qcpgen.small_mixed(0)
    h, t = make_handle(q, max_iter=3, chunk=2, engine=engine)
    dx, dy, ds, info, st = gpu_jvp(h, t)
    assert st == Q.QCPD_WARN_NOT_CONVERGED and info.iters == 3 and (info.flags & 1)


@pytest.mark.parametrize("engine", [Q.QCPD_ENGINE_GRAPH, Q.QCPD_ENGINE_PERSISTENT])
def test_deterministic(engine):
    q = qcpgen.small_mixed(1, n=120, A_density=0.08, P_rank=100, P_eps=0.1)
    h, t = make_handle(q, tol=1e-10, engine=engine)
    a = gpu_jvp(h, t)
    b = gpu_jvp(h, t)
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(u, v)
    c = gpu_vjp(h, t)
    d = gpu_vjp(h, t)
    for u, v in zip(c[:4], d[:4]):
        assert np.array_equal(u, v)


def test_errors_are_reported():
    q = qcpgen.small_mixed(0)
    t = to_device(q)
    cones = cones_of(q)
    # NaN in the data
    bad = t["q"].clone()
    bad[3] = float("nan")
    with pytest.raises(Q.QCPDError) as e:
        Q.qcpd_create(t["P"], t["A"], bad, t["b"], cones, t["x"], t["y"], t["s"])
    assert e.value.status == Q.QCPD_ERR_NAN
    # cone rows do not add up to m
    c2 = Q.Cones(n_zero=cones.n_zero + 1, n_nonneg=cones.n_nonneg, soc=cones.soc,
                 psd=cones.psd, n_exp=cones.n_exp)
    with pytest.raises(Q.QCPDError) as e:
        Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], c2, t["x"], t["y"], t["s"])
    assert e.value.status == Q.QCPD_ERR_CONE
    # asymmetric P
    Pv = t["P"][2].clone()
    Pv[1] += 1.0
    with pytest.raises(Q.QCPDError) as e:
        Q.qcpd_create((t["P"][0], t["P"][1], Pv), t["A"], t["q"], t["b"], cones, t["x"], t["y"], t["s"])
    assert e.value.status == Q.QCPD_ERR_PATTERN
    # column index out of range in A
    Aci = t["A"][1].clone()
    Aci[0] = q.n + 5
    with pytest.raises(Q.QCPDError) as e:
        Q.qcpd_create(t["P"], (t["A"][0], Aci, t["A"][2]), t["q"], t["b"], cones, t["x"], t["y"], t["s"])
    assert e.value.status == Q.QCPD_ERR_INVALID_ARG
    # NaN in a perturbation
    h, _ = make_handle(q)
    dq = t["dq"].clone()
    dq[0] = float("inf")
    with pytest.raises(Q.QCPDError) as e:
        Q.qcpd_jvp(h, t["dP"], t["dA"], dq, t["db"])
    assert e.value.status == Q.QCPD_ERR_NAN
