"""Learned diagonal preconditioner: binding of the feature, inference and training entry
points of include/qcpd.h, and the model container (FP32 parameter blob + JSON metadata).

The model maps each index of z = (x, y, tau) to log corrections of the Jacobi column and row
scales of the LSQR operator; it is trained on the two-sided equilibration scales the library
computes for training problems (qcpd_learned_targets). All arithmetic runs in the HIP
library; this module marshals tensors and keeps the training loop's bookkeeping.
"""
from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import json
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _capi as C
from .api import Handle, QCPDError, _ptr

NFEAT = C.QCPD_NFEAT
NPARAM = C.QCPD_MLP_PARAMS
FEATURE_SCHEMA = [
    "log column norm of F (cone Jacobians replaced by their diagonals)",
    "log row norm of F (same)",
    "kind: x", "kind: zero", "kind: nonneg", "kind: SOC", "kind: PSD", "kind: exp", "kind: tau",
    "diagonal of DPi (1 for x and tau)",
    "log(1 + |P_ii|) (x only)",
    "log(1 + stored entries of the row of [P A'] (x) or A (y))",
]
FORMAT = "qcpd-mlp-v1"


def _lib():
    return C.load()


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check(st: int, where: str):
    if st < 0:
        raise QCPDError(st, where)


def qcpd_features(h: Handle) -> torch.Tensor:
    """Feature rows of the handle's operator: (N, NFEAT) float32 on the handle's device."""
    feat = torch.empty((h.N, NFEAT), dtype=torch.float32, device=h.device)
    with torch.cuda.device(h.device):
        _check(_lib().qcpd_features(h.ptr, _ptr(feat, torch.float32, "feat")), "qcpd_features")
    return feat


def qcpd_learned_targets(h: Handle) -> torch.Tensor:
    """Training targets of the handle: (N, 2) float32, log(equilibration / Jacobi) scales."""
    tgt = torch.empty((h.N, 2), dtype=torch.float32, device=h.device)
    with torch.cuda.device(h.device):
        _check(_lib().qcpd_learned_targets(h.ptr, _ptr(tgt, torch.float32, "target")),
               "qcpd_learned_targets")
    return tgt


def qcpd_set_learned(h: Handle, weights: torch.Tensor):
    """Install the scales the model predicts for this handle (QCPD_PRECOND_LEARNED)."""
    with torch.cuda.device(h.device):
        _check(_lib().qcpd_set_learned(h.ptr, _ptr(weights, torch.float32, "weights", NPARAM)),
               "qcpd_set_learned")


def qcpd_mlp_init(feat: torch.Tensor, seed: int, weights: Optional[torch.Tensor] = None):
    w = weights if weights is not None else torch.empty(NPARAM, dtype=torch.float32,
                                                        device=feat.device)
    with torch.cuda.device(feat.device):
        _check(_lib().qcpd_mlp_init(_ptr(feat, torch.float32, "feat"), int(feat.shape[0]),
                                    ctypes.c_uint64(int(seed)), _ptr(w, torch.float32, "weights",
                                                                     NPARAM),
                                    _stream(feat.device)), "qcpd_mlp_init")
    return w


def qcpd_mlp_predict(feat: torch.Tensor, weights: torch.Tensor) -> torch.Tensor:
    out = torch.empty((feat.shape[0], 2), dtype=torch.float32, device=feat.device)
    with torch.cuda.device(feat.device):
        _check(_lib().qcpd_mlp_predict(_ptr(feat, torch.float32, "feat"), int(feat.shape[0]),
                                       _ptr(weights, torch.float32, "weights", NPARAM),
                                       _ptr(out, torch.float32, "out"), _stream(feat.device)),
               "qcpd_mlp_predict")
    return out


def qcpd_mlp_workspace_floats(nrows: int) -> int:
    return int(_lib().qcpd_mlp_workspace_floats(int(nrows)))


def qcpd_mlp_grad(feat, target, weights, workspace=None, grad=None) -> torch.Tensor:
    """Gradient of the mean squared error (NPARAM + 1 floats; the last is the loss)."""
    nrows = int(feat.shape[0])
    dev = feat.device
    if workspace is None:
        workspace = torch.empty(qcpd_mlp_workspace_floats(nrows), dtype=torch.float32, device=dev)
    if grad is None:
        grad = torch.empty(NPARAM + 1, dtype=torch.float32, device=dev)
    with torch.cuda.device(dev):
        _check(_lib().qcpd_mlp_grad(_ptr(feat, torch.float32, "feat"),
                                    _ptr(target, torch.float32, "target", 2 * nrows), nrows,
                                    _ptr(weights, torch.float32, "weights", NPARAM),
                                    _ptr(workspace, torch.float32, "workspace"),
                                    _ptr(grad, torch.float32, "grad", NPARAM + 1), _stream(dev)),
               "qcpd_mlp_grad")
    return grad


def qcpd_mlp_adam(grad, weights, adam_m, adam_v, step: int, lr: float):
    dev = weights.device
    with torch.cuda.device(dev):
        _check(_lib().qcpd_mlp_adam(_ptr(grad, torch.float32, "grad"),
                                    _ptr(weights, torch.float32, "weights", NPARAM),
                                    _ptr(adam_m, torch.float32, "adam_m", NPARAM),
                                    _ptr(adam_v, torch.float32, "adam_v", NPARAM), int(step),
                                    ctypes.c_float(lr), _stream(dev)), "qcpd_mlp_adam")


@dataclasses.dataclass
class LearnedModel:
    """FP32 parameter blob (NPARAM floats, on a GPU) plus metadata."""
    weights: torch.Tensor
    meta: dict = dataclasses.field(default_factory=dict)

    def install(self, h: Handle):
        qcpd_set_learned(h, self.weights)

    def save(self, path: str):
        """Writes path + '.bin' (little-endian float32) and path + '.json'."""
        blob = self.weights.detach().cpu().numpy().astype("<f4").tobytes()
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path + ".bin", "wb") as f:
            f.write(blob)
        meta = dict(self.meta)
        meta.update(format=FORMAT, nfeat=NFEAT, hidden=C.QCPD_MLP_HIDDEN, params=NPARAM,
                    feature_schema=FEATURE_SCHEMA, sha256=hashlib.sha256(blob).hexdigest())
        with open(path + ".json", "w") as f:
            json.dump(meta, f, indent=1)

    @classmethod
    def load(cls, path: str, device="cuda:0") -> "LearnedModel":
        with open(path + ".json") as f:
            meta = json.load(f)
        if meta.get("format") != FORMAT or meta.get("params") != NPARAM or \
                meta.get("nfeat") != NFEAT:
            raise ValueError(f"{path}: not a {FORMAT} model with {NPARAM} parameters")
        blob = open(path + ".bin", "rb").read()
        if hashlib.sha256(blob).hexdigest() != meta.get("sha256"):
            raise ValueError(f"{path}.bin does not match the checksum in its metadata")
        w = np.frombuffer(blob, dtype="<f4")
        if w.size != NPARAM:
            raise ValueError(f"{path}.bin holds {w.size} floats, expected {NPARAM}")
        return cls(torch.tensor(w.astype(np.float32), device=device), meta)


def train(features: Sequence[torch.Tensor], targets: Sequence[torch.Tensor], *, steps=2000,
          lr=3e-3, lr_final=3e-4, seed=0, log_every=100, log=None) -> LearnedModel:
    """Full-batch Adam on the concatenated rows of all training operators. The learning rate
    decays geometrically from lr to lr_final. Returns the model; meta['loss'] holds
    (step, loss) pairs."""
    feat = torch.cat([f.reshape(-1, NFEAT) for f in features]).contiguous()
    tgt = torch.cat([t.reshape(-1, 2) for t in targets]).contiguous()
    dev = feat.device
    w = qcpd_mlp_init(feat, seed)
    m = torch.zeros(NPARAM, dtype=torch.float32, device=dev)
    v = torch.zeros(NPARAM, dtype=torch.float32, device=dev)
    ws = torch.empty(qcpd_mlp_workspace_floats(feat.shape[0]), dtype=torch.float32, device=dev)
    g = torch.empty(NPARAM + 1, dtype=torch.float32, device=dev)
    history: List[tuple] = []
    decay = (lr_final / lr) ** (1.0 / max(1, steps - 1))
    for step in range(1, steps + 1):
        qcpd_mlp_grad(feat, tgt, w, ws, g)
        qcpd_mlp_adam(g, w, m, v, step, lr * decay ** (step - 1))
        if step == 1 or step % log_every == 0 or step == steps:
            loss = float(g[NPARAM].item())  # loss at the weights before this step
            history.append((step, loss))
            if log:
                log(f"step {step} loss {loss:.5f}")
    final = float(qcpd_mlp_grad(feat, tgt, w, ws, g)[NPARAM].item())
    meta = dict(steps=steps, lr=lr, lr_final=lr_final, seed=seed, rows=int(feat.shape[0]),
                loss=history, final_loss=final)
    return LearnedModel(w, meta)
