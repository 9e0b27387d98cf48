"""torch.autograd integration: the solution map S(theta) = (x, y, s) of a QCP as a
differentiable function of the data theta = (P values, A values, q, b).

The forward pass does not solve the QCP from scratch: as in the paper (Sec. 2.2), the
solution comes from an upstream solver and is passed in. With refine_tol set in the
structure, the point passed in is a warm start (a nearby solution, such as the previous one
when theta moves in a learning loop, Sec. 3.4) that the library refines to a solution of the
current data by Newton steps (qcpd_resolve) before building its handle there. The forward
pass returns the solution and keeps a library handle built at it. The backward pass is the adjoint of the derivative (Sec. 3.2) evaluated by the
HIP library (qcpd_vjp); forward-mode AD (torch.func.jvp / autograd.forward_ad) uses the
derivative itself (Sec. 3.1, qcpd_jvp). Gradients for P and A are on their stored patterns;
the gradient for P is symmetric on the pattern.

batch_solution_map does the same for many problems of uneven sizes at once: the forward pass
builds one batch handle, the backward pass is one qcpd_batch_vjp call (the per-problem
adjoints of all problems in the same launches), forward mode one qcpd_batch_jvp call.
"""
from __future__ import annotations

import dataclasses
import warnings
from typing import Optional, Sequence

import torch

from . import api
from . import batch as B


@dataclasses.dataclass
class QCPStructure:
    """Everything about the problem that is not differentiated: the sparsity patterns (int32
    GPU tensors, P in full symmetric CSR), the cone and the LSQR options."""
    P_rowptr: torch.Tensor
    P_colind: torch.Tensor
    A_rowptr: torch.Tensor
    A_colind: torch.Tensor
    cones: api.Cones
    opts: Optional[api.Opts] = None
    # refine the passed point to a solution of the current data first (None: take it as is)
    refine_tol: Optional[float] = None
    refine_max_newton: int = 20


class _SolutionMap(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P_val, A_val, q, b, x, y, s, structure: QCPStructure):
        st = structure
        ctx.resolve_info = None
        if st.refine_tol is not None:
            x, y, s, info, status = api.qcpd_resolve(
                (st.P_rowptr, st.P_colind, P_val.detach()), (st.A_rowptr, st.A_colind, A_val.detach()),
                q.detach(), b.detach(), st.cones, x.detach(), y.detach(), s.detach(),
                tol=st.refine_tol, max_newton=st.refine_max_newton, opts=st.opts)
            ctx.resolve_info = info
            if status != 0:
                warnings.warn(f"qcpd_resolve: {api.qcpd_status_str(status)} "
                              f"(steps {info.newton_iters}, residual {info.residual:.2e})")
        h = api.qcpd_create((st.P_rowptr, st.P_colind, P_val.detach()),
                            (st.A_rowptr, st.A_colind, A_val.detach()),
                            q.detach(), b.detach(), st.cones, x.detach(), y.detach(), s.detach(),
                            opts=st.opts)
        ctx.handle = h
        return x.detach().clone(), y.detach().clone(), s.detach().clone()

    @staticmethod
    def backward(ctx, gx, gy, gs):
        h = ctx.handle
        f64 = dict(dtype=torch.float64, device=h.device)
        gx = torch.zeros(h.n, **f64) if gx is None else gx.contiguous()
        gy = torch.zeros(h.m, **f64) if gy is None else gy.contiguous()
        gs = torch.zeros(h.m, **f64) if gs is None else gs.contiguous()
        dP, dA, dq, db, info, status = api.qcpd_vjp(h, gx, gy, gs)
        ctx.vjp_info = info
        if status != 0:
            warnings.warn(f"qcpd_vjp: {api.qcpd_status_str(status)} "
                          f"(iters {info.iters}, residual {info.rel_residual:.2e})")
        return dP, dA, dq, db, None, None, None, None

    @staticmethod
    def jvp(ctx, dP, dA, dq, db, dx_in, dy_in, ds_in, _structure):
        h = ctx.handle
        f64 = dict(dtype=torch.float64, device=h.device)
        z = lambda k: torch.zeros(k, **f64)
        dP = z(h.nnzP) if dP is None else dP.contiguous()
        dA = z(h.nnzA) if dA is None else dA.contiguous()
        dq = z(h.n) if dq is None else dq.contiguous()
        db = z(h.m) if db is None else db.contiguous()
        dx, dy, ds, info, status = api.qcpd_jvp(h, dP, dA, dq, db)
        if status != 0:
            warnings.warn(f"qcpd_jvp: {api.qcpd_status_str(status)} "
                          f"(iters {info.iters}, residual {info.rel_residual:.2e})")
        return dx, dy, ds


def qcp_solution_map(P_val, A_val, q, b, x, y, s, structure: QCPStructure):
    """(x, y, s) as a differentiable function of (P_val, A_val, q, b) at a given solution, or
    at the solution refined from the given point when structure.refine_tol is set."""
    return _SolutionMap.apply(P_val, A_val, q, b, x, y, s, structure)


@dataclasses.dataclass
class BatchStructure:
    """The fixed part of a batch of problems: per-problem sizes and cones, and the concatenated
    sparsity patterns (local CSR row pointers and column indices, int32 GPU tensors)."""
    n: Sequence[int]
    m: Sequence[int]
    nnz_P: Sequence[int]
    nnz_A: Sequence[int]
    cones: Sequence[api.Cones]
    P_rowptr: torch.Tensor
    P_colind: torch.Tensor
    A_rowptr: torch.Tensor
    A_colind: torch.Tensor
    opts: Optional[api.Opts] = None
    # the lane schedule of the batch's loop kernels is chosen by the autotuner on the first
    # forward (unless opts fix nnz_per_lane_F or tune is False) and kept for later ones
    tune: bool = True
    tuned: Optional[dict] = None


def _batch_opts(st: BatchStructure, make, device) -> api.Opts:
    opts = st.opts or api.qcpd_opts_default()
    if not st.tune or opts.nnz_per_lane_F > 0:
        return opts
    if st.tuned is None:
        from . import tune as T
        f64 = dict(dtype=torch.float64, device=device)
        g = torch.Generator(device=device).manual_seed(0)
        inputs = (torch.zeros(sum(st.nnz_P), **f64), torch.zeros(sum(st.nnz_A), **f64),
                  torch.randn(sum(st.n), generator=g, **f64), torch.zeros(sum(st.m), **f64))
        h, _, report = T.tune_batch_lanes(make, inputs, opts, cache=T.TuneCache())
        h.close()
        st.tuned = report
    return api.Opts(**{**opts.__dict__, "nnz_per_lane_F": st.tuned["nnz_per_lane"]})


class _BatchSolutionMap(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P_val, A_val, q, b, x, y, s, structure: BatchStructure):
        st = structure

        def make(o):
            return B.qcpd_batch_create(st.n, st.m, st.nnz_P, st.nnz_A, st.cones, st.P_rowptr,
                                       st.P_colind, P_val.detach(), st.A_rowptr, st.A_colind,
                                       A_val.detach(), q.detach(), b.detach(), x.detach(),
                                       y.detach(), s.detach(), opts=o)

        h = make(_batch_opts(st, make, P_val.device))
        ctx.handle = h
        return x.detach().clone(), y.detach().clone(), s.detach().clone()

    @staticmethod
    def backward(ctx, gx, gy, gs):
        h = ctx.handle
        f64 = dict(dtype=torch.float64, device=h.device)
        sn, sm = sum(h.n), sum(h.m)
        gx = torch.zeros(sn, **f64) if gx is None else gx.contiguous()
        gy = torch.zeros(sm, **f64) if gy is None else gy.contiguous()
        gs = torch.zeros(sm, **f64) if gs is None else gs.contiguous()
        dP, dA, dq, db, infos, status = B.qcpd_batch_vjp(h, gx, gy, gs)
        ctx.vjp_infos = infos
        if status != 0:
            bad = [i for i, inf in enumerate(infos) if inf.flags & 1]
            warnings.warn(f"qcpd_batch_vjp: {api.qcpd_status_str(status)} (problems {bad[:8]})")
        return dP, dA, dq, db, None, None, None, None

    @staticmethod
    def jvp(ctx, dP, dA, dq, db, dx_in, dy_in, ds_in, _structure):
        h = ctx.handle
        f64 = dict(dtype=torch.float64, device=h.device)
        z = lambda k: torch.zeros(k, **f64)
        dP = z(sum(h.nnzP)) if dP is None else dP.contiguous()
        dA = z(sum(h.nnzA)) if dA is None else dA.contiguous()
        dq = z(sum(h.n)) if dq is None else dq.contiguous()
        db = z(sum(h.m)) if db is None else db.contiguous()
        dx, dy, ds, infos, status = B.qcpd_batch_jvp(h, dP, dA, dq, db)
        if status != 0:
            warnings.warn(f"qcpd_batch_jvp: {api.qcpd_status_str(status)}")
        return dx, dy, ds


def batch_solution_map(P_val, A_val, q, b, x, y, s, structure: BatchStructure):
    """The concatenated (x, y, s) of every problem of a batch as a differentiable function of
    the concatenated data (P values, A values, q, b) at given solutions."""
    return _BatchSolutionMap.apply(P_val, A_val, q, b, x, y, s, structure)
