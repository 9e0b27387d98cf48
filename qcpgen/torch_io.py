"""Move a generated QCP instance to a GPU as torch tensors (layout only)."""
from __future__ import annotations

import numpy as np
import torch


def to_device(qcp, device="cuda:0"):
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)
    i = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32), device=device)
    return dict(
        P=(i(qcp.P.indptr), i(qcp.P.indices), f(qcp.P.data)),
        A=(i(qcp.A.indptr), i(qcp.A.indices), f(qcp.A.data)),
        q=f(qcp.q), b=f(qcp.b), x=f(qcp.x), y=f(qcp.y), s=f(qcp.s),
        dP=f(qcp.dP), dA=f(qcp.dA), dq=f(qcp.dq), db=f(qcp.db),
        gx=f(qcp.gx), gy=f(qcp.gy), gs=f(qcp.gs),
    )


def cones_of(qcp):
    from paper_2508_17522_amd import Cones
    c = qcp.cones
    return Cones(n_zero=c.n_zero, n_nonneg=c.n_nonneg, soc=list(c.soc), psd=list(c.psd),
                 n_exp=c.n_exp, pow=list(c.pow), dpow=list(c.dpow))


def batch_to_device(qcps, device="cuda:0"):
    """Concatenations of a list of instances, problem after problem (local CSR indices)."""
    f = lambda parts: torch.as_tensor(np.ascontiguousarray(np.concatenate(parts), dtype=np.float64),
                                      device=device)
    i = lambda parts: torch.as_tensor(np.ascontiguousarray(np.concatenate(parts), dtype=np.int32),
                                      device=device)
    out = dict(
        n=[q.n for q in qcps], m=[q.m for q in qcps],
        nnz_P=[q.P.nnz for q in qcps], nnz_A=[q.A.nnz for q in qcps],
        cones=[cones_of(q) for q in qcps],
        P_rowptr=i([q.P.indptr for q in qcps]), P_colind=i([q.P.indices for q in qcps]),
        P_val=f([q.P.data for q in qcps]),
        A_rowptr=i([q.A.indptr for q in qcps]), A_colind=i([q.A.indices for q in qcps]),
        A_val=f([q.A.data for q in qcps]),
    )
    for k in ("q", "b", "x", "y", "s", "dP", "dA", "dq", "db", "gx", "gy", "gs"):
        out[k] = f([getattr(q, k) for q in qcps])
    return out


def batch_create_args(bt):
    return (bt["n"], bt["m"], bt["nnz_P"], bt["nnz_A"], bt["cones"], bt["P_rowptr"],
            bt["P_colind"], bt["P_val"], bt["A_rowptr"], bt["A_colind"], bt["A_val"], bt["q"],
            bt["b"], bt["x"], bt["y"], bt["s"])
