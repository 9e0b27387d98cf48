"""Learned preconditioner on the GPU: the MLP kernels against a plain float64 PyTorch CPU
reference of the same parameter layout, the feature and target rows against host values,
and LSQR with the learned scaling against the oracle (same bar as the other parity tests),
including the fall-back to Jacobi."""
import numpy as np
import pytest
import scipy.sparse as sp

import qcpgen
from oracle import derivative as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2508_17522_amd as Q  # noqa: E402
from paper_2508_17522_amd import learned as L  # noqa: E402
from qcpgen.torch_io import cones_of, to_device  # noqa: E402

F, H = Q._capi.QCPD_NFEAT, Q._capi.QCPD_MLP_HIDDEN
BAR = 1e-7


def unpack(w):
    w = w.detach().double().cpu()
    o = 0

    def take(k, shape=None):
        nonlocal o
        t = w[o:o + k]
        o += k
        return t.view(*shape) if shape else t
    mu, sd = take(F), take(F)
    W1, b1 = take(H * F, (H, F)), take(H)
    W2, b2 = take(H * H, (H, H)), take(H)
    W3, b3 = take(2 * H, (2, H)), take(2)
    assert o == L.NPARAM
    return mu, sd, W1, b1, W2, b2, W3, b3


def ref_forward(params, x):
    mu, sd, W1, b1, W2, b2, W3, b3 = params
    xn = (x - mu) / sd
    h1 = torch.tanh(xn @ W1.T + b1)
    h2 = torch.tanh(h1 @ W2.T + b2)
    return h2 @ W3.T + b3


def random_rows(n, seed):
    g = torch.Generator().manual_seed(seed)
    x = torch.randn(n, F, generator=g, dtype=torch.float64)
    x[:, 2:9] = (torch.rand(n, 7, generator=g) < 0.3).double()
    t = torch.randn(n, 2, generator=g, dtype=torch.float64) * 0.5
    return x, t


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.mark.parametrize("nrows", [1, 37, 1000, 70001])
def test_mlp_predict_and_grad_match_reference(nrows):
    x, t = random_rows(nrows, nrows)
    feat = x.float().cuda().contiguous()
    tgt = t.float().cuda().contiguous()
    w = L.qcpd_mlp_init(feat, seed=7)
    params = unpack(w)
    # init: standardisation from the data, zero biases, Glorot bounds
    xf = feat.double().cpu()
    sd_ref = xf.std(dim=0, unbiased=False)
    assert torch.allclose(params[0], xf.mean(dim=0), rtol=1e-5, atol=1e-5)
    expect_sd = torch.where(sd_ref > 1e-3, sd_ref, torch.ones_like(sd_ref))
    assert torch.allclose(params[1], expect_sd, rtol=1e-4, atol=1e-5)
    for b in (params[3], params[5], params[7]):
        assert torch.all(b == 0)
    assert params[2].abs().max() <= (6.0 / (F + H)) ** 0.5 * (1 + 1e-6)
    assert params[4].abs().max() <= (6.0 / (H + H)) ** 0.5 * (1 + 1e-6)
    # make the biases non-zero so that their gradients are exercised
    with torch.no_grad():
        g = torch.Generator().manual_seed(3)
        off = torch.zeros(L.NPARAM, dtype=torch.float32)
        o = 2 * F + H * F
        off[o:o + H] = 0.1 * torch.randn(H, generator=g)
        o += H + H * H
        off[o:o + H] = 0.1 * torch.randn(H, generator=g)
        o += H + 2 * H
        off[o:o + 2] = torch.tensor([0.3, -0.2])
        w += off.cuda()
    params = unpack(w)
    out = L.qcpd_mlp_predict(feat, w).double().cpu()
    ref = ref_forward(params, xf)
    err = (out - ref).abs().max().item()
    print(f"[mlp nrows={nrows}] predict max abs err {err:.2e}", flush=True)
    assert err <= 1e-4 * (1 + ref.abs().max().item())
    # gradient of the mean squared error
    ps = [p.clone().requires_grad_(True) for p in params]
    loss = ((ref_forward(ps, xf) - tgt.double().cpu()) ** 2).sum() / nrows
    loss.backward()
    gref = torch.cat([torch.zeros(2 * F, dtype=torch.float64)] +
                     [p.grad.reshape(-1) for p in ps[2:]])
    g = L.qcpd_mlp_grad(feat, tgt, w).double().cpu()
    e = rel(g[:L.NPARAM].numpy(), gref.numpy())
    print(f"[mlp nrows={nrows}] grad rel err {e:.2e}, loss {g[L.NPARAM].item():.6f} vs "
          f"{loss.item():.6f}", flush=True)
    assert e <= 1e-4
    assert torch.all(g[:2 * F] == 0)
    assert abs(g[L.NPARAM].item() - loss.item()) <= 1e-4 * (1 + loss.item())


def test_adam_step_matches_reference():
    x, t = random_rows(500, 11)
    feat, tgt = x.float().cuda(), t.float().cuda()
    w = L.qcpd_mlp_init(feat, seed=1)
    m = torch.zeros(L.NPARAM, device="cuda")
    v = torch.zeros(L.NPARAM, device="cuda")
    sl = slice(2 * F, L.NPARAM)
    for step, lr in ((1, 1e-2), (2, 5e-3), (3, 5e-3)):
        g = L.qcpd_mlp_grad(feat, tgt, w)
        gc = g[:L.NPARAM].double().cpu()
        w0, m0, v0 = w.double().cpu(), m.double().cpu(), v.double().cpu()
        L.qcpd_mlp_adam(g, w, m, v, step, lr)
        m1 = 0.9 * m0 + 0.1 * gc
        v1 = 0.999 * v0 + 0.001 * gc ** 2
        w1 = w0 - lr * (m1 / (1 - 0.9 ** step)) / ((v1 / (1 - 0.999 ** step)).sqrt() + 1e-8)
        assert torch.equal(w.double().cpu()[:2 * F], w0[:2 * F])  # mu, sd untouched
        assert (m.double().cpu()[sl] - m1[sl]).abs().max().item() <= 1e-6 * (1 + m1.abs().max().item())
        e = (w.double().cpu()[sl] - w1[sl]).abs().max().item()
        assert e <= 1e-6 + 1e-3 * lr, (step, e)


def test_training_is_deterministic_and_reduces_loss():
    x, t = random_rows(5000, 5)
    tgt = (torch.tanh(x[:, :2]) * 0.7 + 0.1 * x[:, 2:4]).float().cuda()
    feat = x.float().cuda()
    m1 = L.train([feat], [tgt], steps=200, lr=1e-2, lr_final=1e-3, seed=3, log_every=50)
    m2 = L.train([feat], [tgt], steps=200, lr=1e-2, lr_final=1e-3, seed=3, log_every=50)
    assert torch.equal(m1.weights, m2.weights)
    first, last = m1.meta["loss"][0][1], m1.meta["final_loss"]
    print(f"[train] loss {first:.4f} -> {last:.5f}", flush=True)
    assert last < 0.1 * first


def handle(qcp, tol=1e-12, precond=Q.QCPD_PRECOND_JACOBI, max_iter=0):
    t = to_device(qcp)
    o = Q.Opts(tol=tol, precond=precond, max_iter=max_iter)
    return Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones_of(qcp), t["x"], t["y"], t["s"],
                         opts=o), t


def test_features_and_targets_match_host_values():
    qcp = qcpgen.small_mixed(1)
    h, _ = handle(qcp)
    feat = L.qcpd_features(h).double().cpu().numpy()
    tgt = L.qcpd_learned_targets(h).double().cpu().numpy()
    dg = Q.qcpd_get_diagnostics(h)
    jc, jr = dg["jacobi_jvp"].cpu().numpy(), dg["jacobi_vjp"].cpu().numpy()
    ec, er = dg["equil_col"].cpu().numpy(), dg["equil_row"].cpu().numpy()
    jd = dg["jdiag"].cpu().numpy()
    n, m = qcp.n, qcp.m
    K = qcp.cones
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    assert np.array_equal(feat[:, 0], f32(-np.log(jc)))
    assert np.array_equal(feat[:, 1], f32(-np.log(jr)))
    # one-hot kinds
    kinds = np.zeros(n + m + 1, dtype=int)
    kinds[:n] = 0
    r = n
    spans = [(K.n_zero, 1), (K.n_nonneg, 2), (sum(K.soc), 3),
             (sum(k * (k + 1) // 2 for k in K.psd), 4), (3 * K.n_exp, 5)]
    for cnt, kd in spans:
        kinds[r:r + cnt] = kd
        r += cnt
    kinds[-1] = 6
    assert r == n + m
    onehot = np.eye(7)[kinds]
    assert np.array_equal(feat[:, 2:9], onehot)
    Pd = sp.csr_matrix(qcp.P).diagonal()
    A = sp.csr_matrix(qcp.A)
    Pnnz = np.diff(sp.csr_matrix(qcp.P).indptr)
    Acol = np.diff(A.tocsc().indptr)
    Arow = np.diff(A.indptr)
    assert np.array_equal(feat[:n, 9], np.ones(n))
    assert np.array_equal(feat[n:n + m, 9], f32(jd))
    assert feat[-1, 9] == 1.0
    assert np.array_equal(feat[:n, 10], f32(np.log1p(np.abs(Pd))))
    assert np.all(feat[n:, 10] == 0)
    assert np.array_equal(feat[:n, 11], f32(np.log1p(Pnnz + Acol)))
    assert np.array_equal(feat[n:n + m, 11], f32(np.log1p(Arow)))
    assert feat[-1, 11] == np.float32(np.log1p(n + m))
    assert np.array_equal(tgt[:, 0], f32(np.log(ec / jc)))
    assert np.array_equal(tgt[:, 1], f32(np.log(er / jr)))
    h.close()


def _check_against_oracle(qcp, h, t, expect_fallback):
    dx, dy, ds, info, st = Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"])
    print(f"[{qcp.name}] learned jvp iters={info.iters} flags={info.flags} "
          f"rel_res={info.rel_residual:.2e}", flush=True)
    assert st == Q.QCPD_OK
    assert bool(info.flags & Q.QCPD_FLAG_FALLBACK) == expect_fallback
    ref = D.jvp_dense(qcp, qcp.dP, qcp.dA, qcp.dq, qcp.db)
    errs = [rel(a.cpu().numpy(), b) for a, b in zip((dx, dy, ds), ref)]
    assert max(errs) <= BAR, errs
    dP, dA, dq, db, info2, st2 = Q.qcpd_vjp(h, t["gx"], t["gy"], t["gs"])
    print(f"[{qcp.name}] learned vjp iters={info2.iters} flags={info2.flags} "
          f"rel_res={info2.rel_residual:.2e}", flush=True)
    assert st2 == Q.QCPD_OK
    assert bool(info2.flags & Q.QCPD_FLAG_FALLBACK) == expect_fallback
    refv = D.vjp_dense(qcp, qcp.gx, qcp.gy, qcp.gs)
    errs2 = [rel(a.cpu().numpy(), b) for a, b in zip((dP, dA, dq, db), refv)]
    assert max(errs2) <= BAR, errs2


def test_learned_scaling_matches_oracle():
    train_qcps = [qcpgen.small_mixed(i) for i in (2, 3, 4)]
    feats, tgts = [], []
    for q in train_qcps:
        h, _ = handle(q)
        feats.append(L.qcpd_features(h))
        tgts.append(L.qcpd_learned_targets(h))
        h.close()
    model = L.train(feats, tgts, steps=400, lr=1e-2, lr_final=1e-3, seed=0)
    qcp = qcpgen.small_mixed(0)
    h, t = handle(qcp, precond=Q.QCPD_PRECOND_LEARNED)
    with pytest.raises(Q.QCPDError):  # LEARNED without an installed model
        Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"])
    model.install(h)
    _check_against_oracle(qcp, h, t, expect_fallback=False)
    h.close()


def test_learned_falls_back_to_jacobi():
    """A model whose corrections spread the scales over e^+-30 leaves LSQR unable to reach
    the tolerance in FP64; the call must still return the Jacobi-preconditioned result."""
    qcp = qcpgen.small_mixed(0)
    h, t = handle(qcp, precond=Q.QCPD_PRECOND_LEARNED)
    feat = L.qcpd_features(h)
    w = L.qcpd_mlp_init(feat, seed=5)
    with torch.no_grad():
        w[2 * F:] *= 60.0
    L.qcpd_set_learned(h, w)
    _check_against_oracle(qcp, h, t, expect_fallback=True)
    h.close()
