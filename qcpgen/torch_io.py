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
                 n_exp=c.n_exp)
