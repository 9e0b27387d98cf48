"""qcpd_mlp_grad_noalloc (the gradient of the learned-preconditioner loss with its workspace in
a fixed array inside the library) against qcpd_mlp_grad with a caller-allocated workspace,
through the raw C-ABI: two calls in a row, the second on fewer rows, each identical to the
allocating entry point (same kernels, same summation order). Also the argument checks."""
import ctypes

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_17522_amd import _capi as C  # noqa: E402

NP = C.QCPD_MLP_PARAMS


def rows(nrows, seed):
    g = torch.Generator().manual_seed(seed)
    feat = torch.randn(nrows, C.QCPD_NFEAT, generator=g, dtype=torch.float32)
    feat[:, 2:9] = (torch.rand(nrows, 7, generator=g) < 0.3).float()
    tgt = 0.5 * torch.randn(nrows, 2, generator=g, dtype=torch.float32)
    return feat.cuda().contiguous(), tgt.cuda().contiguous()


def grad_alloc(lib, feat, tgt, w, stream):
    n = feat.shape[0]
    ws = torch.empty(int(lib.qcpd_mlp_workspace_floats(n)), dtype=torch.float32, device="cuda")
    g = torch.full((NP + 1,), float("nan"), dtype=torch.float32, device="cuda")
    st = lib.qcpd_mlp_grad(feat.data_ptr(), tgt.data_ptr(), n, w.data_ptr(), ws.data_ptr(),
                           g.data_ptr(), stream)
    assert st == C.QCPD_OK
    return g


def grad_noalloc(lib, feat, tgt, w, stream):
    n = feat.shape[0]
    g = torch.full((NP + 1,), float("nan"), dtype=torch.float32, device="cuda")
    st = lib.qcpd_mlp_grad_noalloc(feat.data_ptr(), tgt.data_ptr(), n, w.data_ptr(),
                                   g.data_ptr(), stream)
    assert st == C.QCPD_OK, st
    return g


def test_noalloc_grad_equals_workspace_grad_on_two_calls():
    lib = C.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    w = torch.empty(NP, dtype=torch.float32, device="cuda")
    # the larger call first (all 256 partial rows of the array in use), then a smaller one
    # that uses fewer rows: stale partials of the first call must not leak into the second
    for nrows, seed in ((70001, 1), (777, 2)):
        feat, tgt = rows(nrows, seed)
        assert lib.qcpd_mlp_init(feat.data_ptr(), nrows, 11, w.data_ptr(), stream) == C.QCPD_OK
        g_ref = grad_alloc(lib, feat, tgt, w, stream)
        g_new = grad_noalloc(lib, feat, tgt, w, stream)
        torch.cuda.synchronize()
        assert torch.isfinite(g_ref).all()
        assert torch.equal(g_new, g_ref), (nrows, (g_new - g_ref).abs().max().item())
        assert g_new[NP].item() > 0.0   # the loss


def test_noalloc_rejects_bad_arguments():
    lib = C.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    feat, tgt = rows(8, 3)
    w = torch.zeros(NP, dtype=torch.float32, device="cuda")
    g = torch.zeros(NP + 1, dtype=torch.float32, device="cuda")
    assert lib.qcpd_mlp_grad_noalloc(feat.data_ptr(), tgt.data_ptr(), 0, w.data_ptr(),
                                     g.data_ptr(), stream) == C.QCPD_ERR_INVALID_ARG
    assert lib.qcpd_mlp_grad_noalloc(None, tgt.data_ptr(), 8, w.data_ptr(),
                                     g.data_ptr(), stream) == C.QCPD_ERR_INVALID_ARG
    assert lib.qcpd_mlp_grad_noalloc(feat.data_ptr(), tgt.data_ptr(), 8, w.data_ptr(),
                                     None, stream) == C.QCPD_ERR_INVALID_ARG
