"""GPU: the library's Jacobi scales and Jacobian diagonal against the oracle, and the
failure paths that the host can force.

* Jacobi scales (column norms of F and of F' with each cone block's Jacobian replaced by its
  diagonal; the right preconditioner of the plain method and the reference of every
  comparison) against the oracle's closed forms, which a CPU test pins to dense norms.
* Points on a kink of a cone projection (App. A: nonnegative z = 0, second-order cone with
  ||u|| = |t|, PSD with a zero eigenvalue) are reported as QCPD_WARN_NONDIFF and the flag is
  carried into every later call's info.
* Inconsistent dimensions (QCPD_ERR_DIM) through the raw C-ABI.
* A point where the reduced KKT matrix is singular (two identical active constraints): the
  derivative does not exist, the least-squares system is inconsistent and the call reports
  QCPD_WARN_NOT_CONVERGED.
"""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

import qcpgen
from oracle import derivative as D
from oracle import embedding as E

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2508_17522_amd as Q  # noqa: E402
from paper_2508_17522_amd import _capi  # noqa: E402
from qcpgen.torch_io import cones_of, to_device  # noqa: E402


def medium():
    return qcpgen.small_mixed(1, n=301, n_zero=37, n_nonneg=260, soc=(3, 4, 5, 6, 7, 8) * 5,
                              psd=(4, 7, 12, 9), n_exp=23, A_density=0.04, P_rank=150,
                              nonneg_active=100)


def create(q, **kw):
    t = to_device(q)
    o = Q.Opts(**kw) if kw else None
    h = Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones_of(q), t["x"], t["y"], t["s"], opts=o)
    return h, t


@pytest.mark.parametrize("which", ["tiny", "small", "medium", "mixed_full"])
def test_jacobi_scales_and_jacobian_diagonal_match_oracle(which):
    q = {"tiny": lambda: qcpgen.tiny_qp(0), "small": lambda: qcpgen.small_mixed(0),
         "medium": medium, "mixed_full": lambda: qcpgen.mixed_qcp(0)}[which]()
    print(f"[{q.name}] n={q.n} m={q.m}", flush=True)
    h, _ = create(q)
    dg = Q.qcpd_get_diagnostics(h)
    emb = E.Embedding(q)
    for key, ref in (("jacobi_jvp", D.jacobi_scale_F(emb)), ("jacobi_vjp", D.jacobi_scale_FT(emb)),
                     ("jdiag", emb.J.diagonal())):
        got = dg[key].cpu().numpy()
        err = np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300 if key != "jdiag" else 1.0))
        print(f"[{q.name}] {key}: max relative difference {err:.2e}", flush=True)
        assert err <= 1e-12
    h.close()


# ---- kinks ------------------------------------------------------------------------------

def _refresh(q):
    """b and q recomputed so that (x, y, s) solves the edited instance exactly."""
    q.b = q.A @ q.x + q.s
    q.q = -(q.P @ q.x) - q.A.T @ q.y
    return q


def kink_nonneg():
    q = qcpgen.tiny_qp(0)
    nz = q.cones.n_zero
    i = nz + int(np.nonzero(q.y[nz:] == 0.0)[0][0])   # an inactive row: s > 0, y = 0
    q.s = q.s.copy()
    q.s[i] = 0.0                                       # z = y - s = 0: kink of the orthant
    return _refresh(q)


def kink_soc():
    q = qcpgen.small_mixed(0)                          # SOC dims (3, 4, 5); the third is a
    r = q.cones.n_zero + q.cones.n_nonneg + 3 + 4      # boundary pair (s, y both on the boundary)
    q.s = q.s.copy()
    q.s[r:r + 5] = 0.0                                 # z = y: ||u|| = t
    return _refresh(q)


def kink_psd():
    q = qcpgen.small_mixed(0)                          # PSD orders (2, 3, 4)
    r = q.cones.n_zero + q.cones.n_nonneg + sum(q.cones.soc) + 3 + 6
    S = qcpgen.smat(q.s[r:r + 10], 4)
    w, V = np.linalg.eigh(S)
    j = int(np.argmax(w > 1e-12))                      # smallest positive eigenvalue of S
    w[j] = 0.0
    q.s = q.s.copy()
    q.s[r:r + 10] = qcpgen.svec((V * w) @ V.T)         # z = Y - S has a zero eigenvalue
    return _refresh(q)


@pytest.mark.parametrize("maker", [kink_nonneg, kink_soc, kink_psd])
def test_kink_is_reported(maker):
    q = maker()
    t = to_device(q)
    h = Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones_of(q), t["x"], t["y"], t["s"],
                      opts=Q.Opts(tol=1e-10))
    print(f"[{maker.__name__}] create status {h.create_status}", flush=True)
    assert h.create_status == Q.QCPD_WARN_NONDIFF
    dx, dy, ds, info, st = Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"])
    print(f"[{maker.__name__}] jvp status {st} flags {info.flags} iters {info.iters}", flush=True)
    assert info.flags & 2
    h.close()


def test_kink_free_instance_is_not_flagged():
    h, _ = create(qcpgen.small_mixed(0))
    assert h.create_status == Q.QCPD_OK
    h.close()


# ---- dimensions ---------------------------------------------------------------------------

def test_inconsistent_dimensions_through_the_c_abi():
    q = qcpgen.small_mixed(0)
    t = to_device(q)
    lib = _capi.load()
    cones = cones_of(q)
    soc = (ctypes.c_int32 * len(cones.soc))(*cones.soc)
    psd = (ctypes.c_int32 * len(cones.psd))(*cones.psd)
    K = _capi.qcpd_cones(cones.n_zero, cones.n_nonneg, len(cones.soc), soc, len(cones.psd), psd,
                         cones.n_exp)

    def csr(tr, nrows, ncols):
        return _capi.qcpd_csr(nrows, ncols, int(tr[1].numel()), ctypes.c_void_p(tr[0].data_ptr()),
                              ctypes.c_void_p(tr[1].data_ptr()), ctypes.c_void_p(tr[2].data_ptr()))

    p = lambda x: ctypes.c_void_p(x.data_ptr())
    for Pc, Ac in ((csr(t["P"], q.n, q.n + 1), csr(t["A"], q.m, q.n)),    # P not square
                   (csr(t["P"], q.n, q.n), csr(t["A"], q.m, q.n - 1))):   # A's columns != n
        h = ctypes.c_void_p()
        st = lib.qcpd_create(ctypes.byref(h), ctypes.byref(Pc), ctypes.byref(Ac), p(t["q"]),
                             p(t["b"]), ctypes.byref(K), p(t["x"]), p(t["y"]), p(t["s"]), None,
                             None)
        assert st == Q.QCPD_ERR_DIM and not h.value


# ---- singular reduced KKT matrix --------------------------------------------------------------

def singular_instance():
    """A copy of a tiny QP whose two active nonnegative rows are made identical: the active
    constraints are dependent, the reduced KKT matrix is singular and the solution map has
    no derivative at this point."""
    q = qcpgen.tiny_qp(0)
    nz = q.cones.n_zero
    act = nz + np.nonzero(q.y[nz:] > 0.0)[0]
    i, j = int(act[0]), int(act[1])
    A = q.A.tolil()
    A[j, :] = A[i, :]
    A = sp.csr_matrix(A)
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    q.A = A
    rng = np.random.default_rng(7)
    q.dA = 1e-2 * rng.standard_normal(A.nnz)
    return _refresh(q)


def test_singular_point_reports_not_converged():
    q = singular_instance()
    c = D.kred_cond(q)
    print(f"oracle cond(K_red) = {c:.2e}", flush=True)
    assert c > 1e14
    h, t = create(q, tol=1e-10, max_iter=4000, graph_chunk=64)
    dx, dy, ds, info, st = Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"])
    print(f"singular: jvp status {st} iters {info.iters} rel residual {info.rel_residual:.2e}",
          flush=True)
    assert st == Q.QCPD_WARN_NOT_CONVERGED and (info.flags & 1)
    assert info.rel_residual > 1e-10
    h.close()
