"""Python binding of the batched C-ABI (qcpd_batch_*): many QCPs of uneven sizes, each with
its own LSQR, evaluated in one launch. Argument marshalling only.

Data are concatenations, problem after problem, of GPU tensors: CSR row pointers are each
problem's local ones (n_i + 1, resp. m_i + 1 entries, starting at 0) with local column
indices; vectors are stacked.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import torch

from . import _capi as C
from .api import Cones, Info, Opts, QCPDError, _lib, _ptr, qcpd_opts_default


class BatchHandle:
    def __init__(self, ptr, n, m, nnzP, nnzA, device, stream):
        self.ptr = ptr
        self.n, self.m, self.nnzP, self.nnzA = list(n), list(m), list(nnzP), list(nnzA)
        self.device = device
        self.stream = stream
        self.create_status = 0

    @property
    def nprob(self):
        return len(self.n)

    def close(self):
        if self.ptr:
            _lib().qcpd_batch_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def qcpd_batch_create(n: Sequence[int], m: Sequence[int], nnz_P: Sequence[int],
                      nnz_A: Sequence[int], cones: Sequence[Cones], P_rowptr, P_colind, P_val,
                      A_rowptr, A_colind, A_val, q, b, x, y, s, opts: Optional[Opts] = None,
                      stream=None) -> BatchHandle:
    B = len(n)
    I32 = C.c_int32 * B
    keep = []
    cone_arr = (C.qcpd_cones * B)()
    for i, c in enumerate(cones):
        cone_arr[i], arrays = c.to_c()
        keep.append(arrays)
    L = C.qcpd_batch_layout(B, I32(*n), I32(*m), I32(*nnz_P), I32(*nnz_A), cone_arr)
    o = (opts or qcpd_opts_default()).to_c()
    dev = q.device
    strm = stream if stream is not None else torch.cuda.current_stream(dev)
    h = ctypes.c_void_p()
    sn, sm, sp, sa = sum(n), sum(m), sum(nnz_P), sum(nnz_A)
    i32, f64 = torch.int32, torch.float64
    with torch.cuda.device(dev):
        st = _lib().qcpd_batch_create(
            ctypes.byref(h), ctypes.byref(L),
            _ptr(P_rowptr, i32, "P_rowptr", sn + B), _ptr(P_colind, i32, "P_colind", sp),
            _ptr(P_val, f64, "P_val", sp), _ptr(A_rowptr, i32, "A_rowptr", sm + B),
            _ptr(A_colind, i32, "A_colind", sa), _ptr(A_val, f64, "A_val", sa),
            _ptr(q, f64, "q", sn), _ptr(b, f64, "b", sm), _ptr(x, f64, "x", sn),
            _ptr(y, f64, "y", sm), _ptr(s, f64, "s", sm), ctypes.byref(o),
            ctypes.c_void_p(strm.cuda_stream))
    del keep
    if st < 0:
        raise QCPDError(st, "qcpd_batch_create")
    out = BatchHandle(h, n, m, nnz_P, nnz_A, dev, strm)
    out.create_status = st
    return out


def _infos(B):
    return (C.qcpd_info * B)()


def qcpd_batch_jvp(h: BatchHandle, dP, dA, dq, db, dx=None, dy=None, ds=None):
    """Returns (dx, dy, ds, [Info] per problem, status)."""
    f64 = dict(dtype=torch.float64, device=h.device)
    sn, sm = sum(h.n), sum(h.m)
    dx = torch.empty(sn, **f64) if dx is None else dx
    dy = torch.empty(sm, **f64) if dy is None else dy
    ds = torch.empty(sm, **f64) if ds is None else ds
    info = _infos(h.nprob)
    with torch.cuda.device(h.device):
        st = _lib().qcpd_batch_jvp(h.ptr, _ptr(dP, torch.float64, "dP", sum(h.nnzP)),
                                   _ptr(dA, torch.float64, "dA", sum(h.nnzA)),
                                   _ptr(dq, torch.float64, "dq", sn), _ptr(db, torch.float64, "db", sm),
                                   _ptr(dx, torch.float64, "dx", sn), _ptr(dy, torch.float64, "dy", sm),
                                   _ptr(ds, torch.float64, "ds", sm), info)
    if st < 0:
        raise QCPDError(st, "qcpd_batch_jvp")
    return dx, dy, ds, [Info.from_c(i) for i in info], st


def qcpd_batch_vjp(h: BatchHandle, gx, gy, gs, dP=None, dA=None, dq=None, db=None):
    """Returns (dP, dA, dq, db, [Info] per problem, status)."""
    f64 = dict(dtype=torch.float64, device=h.device)
    sn, sm = sum(h.n), sum(h.m)
    dP = torch.empty(sum(h.nnzP), **f64) if dP is None else dP
    dA = torch.empty(sum(h.nnzA), **f64) if dA is None else dA
    dq = torch.empty(sn, **f64) if dq is None else dq
    db = torch.empty(sm, **f64) if db is None else db
    info = _infos(h.nprob)
    with torch.cuda.device(h.device):
        st = _lib().qcpd_batch_vjp(h.ptr, _ptr(gx, torch.float64, "gx", sn),
                                   _ptr(gy, torch.float64, "gy", sm), _ptr(gs, torch.float64, "gs", sm),
                                   _ptr(dP, torch.float64, "dP", sum(h.nnzP)),
                                   _ptr(dA, torch.float64, "dA", sum(h.nnzA)),
                                   _ptr(dq, torch.float64, "dq", sn), _ptr(db, torch.float64, "db", sm),
                                   info)
    if st < 0:
        raise QCPDError(st, "qcpd_batch_vjp")
    return dP, dA, dq, db, [Info.from_c(i) for i in info], st


def qcpd_batch_set_opts(h: BatchHandle, opts: Opts):
    o = opts.to_c()
    st = _lib().qcpd_batch_set_opts(h.ptr, ctypes.byref(o))
    if st < 0:
        raise QCPDError(st, "qcpd_batch_set_opts")


def qcpd_batch_set_launch(h: BatchHandle, grid: int = 0):
    """Persistent workgroups of the batch kernel (0 = default: all that fit)."""
    st = _lib().qcpd_batch_set_launch(h.ptr, int(grid))
    if st < 0:
        raise QCPDError(st, "qcpd_batch_set_launch")


def qcpd_batch_get_launch(h: BatchHandle):
    """(grid, default grid)."""
    out = (C.c_int32 * 2)()
    st = _lib().qcpd_batch_get_launch(h.ptr, out)
    if st < 0:
        raise QCPDError(st, "qcpd_batch_get_launch")
    return tuple(out)


def qcpd_batch_destroy(h: BatchHandle):
    h.close()
