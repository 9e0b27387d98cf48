"""The LSQR loop with the input's x part staged in LDS (one workgroup per CU; the CSR sums
with P and A gather from LDS; the cones of the product with F' in a second launch that reads
their raw rows from a buffer, PSD cones of order 33-64 with at most 16 eigenvalues on one
side of zero through the low-rank form of their Jacobian), forced on problems small enough
for the dense oracle: JVP and VJP against its implicit-function solve (relative error <= 1e-7
at tolerance 1e-12) with every cone type, both sides of the low-rank form (smaller sides of
2 to 15 eigenvalues, orders 34 to 60), LSQR and LSMR,
the default launch shape and one with far fewer workgroups than row blocks, a problem
without cone units, and a reduced instance of the n = 20 000 workload's shape. The
full-size workload runs this layout by default (its own tests)."""
import numpy as np
import pytest

import qcpgen
from oracle import derivative as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2508_17522_amd as Q  # noqa: E402
from qcpgen.torch_io import cones_of, to_device  # noqa: E402

BAR = 1e-7


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def medium():
    rng = np.random.default_rng(11)
    return qcpgen.small_mixed(2, n=301, n_zero=37, n_nonneg=260, soc=(3, 4, 5, 6, 7, 8) * 5,
                              psd=(4, 7, 12, 9, 40), n_exp=23, A_density=0.04, P_rank=150,
                              P_eps=1e-2, nonneg_active=60, psd_ranks=(2, 3, 6, 4, 8),
                              pow_alphas=tuple(rng.uniform(0.1, 0.9, 6)),
                              dpow_alphas=tuple(rng.uniform(0.1, 0.9, 4)))


def psd_negative_side():
    """An order-34 PSD cone with 22 positive eigenvalues at the solution: the low-rank
    Jacobian works on the 12 negative ones (J = X minus the low-rank sum)."""
    rng = np.random.default_rng(11)
    return qcpgen.small_mixed(2, n=600, n_zero=37, n_nonneg=260, soc=(3, 4, 5, 6, 7, 8) * 5,
                              psd=(4, 34), n_exp=23, A_density=0.04, P_rank=150, P_eps=1e-2,
                              nonneg_active=10, psd_ranks=(2, 22),
                              pow_alphas=tuple(rng.uniform(0.1, 0.9, 6)),
                              dpow_alphas=tuple(rng.uniform(0.1, 0.9, 4)))


def psd_wide_side(order, ranks, n):
    """One PSD cone of order 53-64 (padded order 64, sums over all 16 k-steps) whose smaller
    side holds 13-16 eigenvalues: the low-rank Jacobian's symmetric product over its whole
    32-column panel."""
    rng = np.random.default_rng(11)
    return qcpgen.small_mixed(3, n=n, n_zero=37, n_nonneg=260, soc=(3, 4, 5, 6, 7, 8) * 5,
                              psd=(4, order), n_exp=23, A_density=0.04, P_rank=150,
                              P_eps=1e-2, nonneg_active=10, psd_ranks=ranks,
                              pow_alphas=tuple(rng.uniform(0.1, 0.9, 6)),
                              dpow_alphas=tuple(rng.uniform(0.1, 0.9, 4)))


CASES = {
    "small": lambda: qcpgen.small_mixed(0),
    "medium": medium,
    "psd_negative_side": psd_negative_side,
    "tiny_qp": lambda: qcpgen.tiny_qp(1),   # zero and nonnegative rows only: no cone launch
    "reduced_large": lambda: qcpgen.large_psd_soc(0, scale=0.04),
    "psd60_positive_15": lambda: psd_wide_side(60, (2, 15), 900),
    "psd53_negative_13": lambda: psd_wide_side(53, (2, 40), 1500),
}


def handle(q, staged=Q.QCPD_CHOICE_ON, **kw):
    t = to_device(q)
    h = Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones_of(q), t["x"], t["y"], t["s"],
                      opts=Q.Opts(staged=staged, **kw))
    return h, t


def check(h, t, q, tag):
    dx, dy, ds, info, st = Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"])
    print(f"[{tag}] jvp iters={info.iters} rel={info.rel_residual:.2e} st={st}", flush=True)
    assert st == Q.QCPD_OK
    ref = D.jvp_dense(q, q.dP, q.dA, q.dq, q.db)
    errs = [rel(a.cpu().numpy(), b) for a, b in zip((dx, dy, ds), ref)]
    dP, dA, dq, db, info2, st2 = Q.qcpd_vjp(h, t["gx"], t["gy"], t["gs"])
    print(f"[{tag}] vjp iters={info2.iters} rel={info2.rel_residual:.2e} st={st2}", flush=True)
    assert st2 == Q.QCPD_OK
    refv = D.vjp_dense(q, q.gx, q.gy, q.gs)
    errs += [rel(a.cpu().numpy(), b) for a, b in zip((dP, dA, dq, db), refv)]
    print(f"[{tag}] errors dx dy ds dP dA dq db {['%.1e' % e for e in errs]}", flush=True)
    assert max(errs) <= BAR


@pytest.mark.parametrize("case,precond,solver", [
    ("small", Q.QCPD_PRECOND_JACOBI, Q.QCPD_SOLVER_LSQR),
    ("medium", Q.QCPD_PRECOND_EQUIL, Q.QCPD_SOLVER_LSQR),
    ("medium", Q.QCPD_PRECOND_EQUIL, Q.QCPD_SOLVER_LSMR),
    ("psd_negative_side", Q.QCPD_PRECOND_EQUIL, Q.QCPD_SOLVER_LSQR),
    ("tiny_qp", Q.QCPD_PRECOND_JACOBI, Q.QCPD_SOLVER_LSQR),
    ("reduced_large", Q.QCPD_PRECOND_EQUIL, Q.QCPD_SOLVER_LSQR),
    ("psd60_positive_15", Q.QCPD_PRECOND_EQUIL, Q.QCPD_SOLVER_LSQR),
    ("psd53_negative_13", Q.QCPD_PRECOND_EQUIL, Q.QCPD_SOLVER_LSQR),
])
def test_staged_loop_matches_dense_oracle(case, precond, solver):
    q = CASES[case]()
    h, t = handle(q, tol=1e-12, precond=precond, solver=solver)
    lay = Q.qcpd_get_layout(h)
    print(f"[{case}] layout {lay} launch {Q.qcpd_get_launch(h)}", flush=True)
    assert lay["staged"] == 1 and lay["psd_split"] == 0
    check(h, t, q, case)
    h.close()


def test_staged_loop_with_few_workgroups():
    """Three workgroups for the F product and two for F': each wave walks many row blocks."""
    q = medium()
    h, t = handle(q, tol=1e-12, precond=Q.QCPD_PRECOND_EQUIL, graph_chunk=5)
    Q.qcpd_set_launch(h, 3, 2)
    assert Q.qcpd_get_launch(h)[:2] == (3, 2)
    check(h, t, q, "medium, grids 3 / 2")
    h.close()


def test_staged_matches_unstaged_and_auto_choice():
    """The same solve with and without staging (different summation orders only), and the
    automatic choice: off on a small problem, on at the full n = 20 000 workload's shape
    (checked through the layout query only; its solves are covered elsewhere)."""
    q = CASES["reduced_large"]()
    out = {}
    for staged in (Q.QCPD_CHOICE_ON, Q.QCPD_CHOICE_OFF):
        h, t = handle(q, staged=staged, tol=1e-12, precond=Q.QCPD_PRECOND_EQUIL)
        j = Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"])
        out[staged] = [x.cpu().numpy() for x in j[:3]]
        assert Q.qcpd_get_layout(h)["staged"] == (1 if staged == Q.QCPD_CHOICE_ON else 0)
        h.close()
    d = max(rel(a, b) for a, b in zip(out[Q.QCPD_CHOICE_ON], out[Q.QCPD_CHOICE_OFF]))
    print(f"staged vs unstaged: largest relative difference {d:.2e}", flush=True)
    assert d <= 1e-8
    h, _ = handle(qcpgen.small_mixed(0), staged=Q.QCPD_CHOICE_AUTO)
    assert Q.qcpd_get_layout(h)["staged"] == 0
    h.close()
    big = qcpgen.large_psd_soc(0)
    h, _ = handle(big, staged=Q.QCPD_CHOICE_AUTO)
    lay = Q.qcpd_get_layout(h)
    print(f"n = 20 000 layout {lay} launch {Q.qcpd_get_launch(h)}", flush=True)
    assert lay["staged"] == 1
    h.close()


def test_layout_options_are_fixed_at_create():
    q = qcpgen.small_mixed(0)
    h, _ = handle(q, staged=Q.QCPD_CHOICE_OFF)
    with pytest.raises(Q.QCPDError) as e:
        Q.qcpd_set_opts(h, Q.Opts(staged=Q.QCPD_CHOICE_ON))
    assert e.value.status == Q.QCPD_ERR_INVALID_ARG
    Q.qcpd_set_opts(h, Q.Opts(staged=Q.QCPD_CHOICE_OFF, tol=1e-10))   # other fields may change
    h.close()
