"""Python binding of the C-ABI: the same entry points as include/qcpd.h, taking torch
tensors that live on the GPU. Argument marshalling only; every step of the computation
runs in the HIP library.

Tensors: float64 for values, int32 for CSR index arrays, contiguous, on a HIP device.
Streams: the handle is bound to torch.cuda.current_stream() at create time unless a stream
is passed.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence

import torch

from . import _capi as C


class QCPDError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {qcpd_status_str(status)} (status {status})")


def _lib():
    return C.load()


def _ptr(t: Optional[torch.Tensor], dtype, name: str, numel: Optional[int] = None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: must be a GPU tensor (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr()) if t.numel() > 0 else ctypes.c_void_p(t.data_ptr() or 0)


@dataclasses.dataclass
class Cones:
    n_zero: int = 0
    n_nonneg: int = 0
    soc: Sequence[int] = ()
    psd: Sequence[int] = ()
    n_exp: int = 0
    pow: Sequence[float] = ()    # exponent of each power cone
    dpow: Sequence[float] = ()   # exponent of each dual power cone

    @property
    def m(self) -> int:
        return (self.n_zero + self.n_nonneg + sum(self.soc)
                + sum(k * (k + 1) // 2 for k in self.psd) + 3 * self.n_exp
                + 3 * len(self.pow) + 3 * len(self.dpow))

    def to_c(self):
        """The C struct and the arrays it points into (keep both alive during the call)."""
        soc = (C.c_int32 * max(len(self.soc), 1))(*self.soc)
        psd = (C.c_int32 * max(len(self.psd), 1))(*self.psd)
        pw = (C.c_double * max(len(self.pow), 1))(*self.pow)
        dp = (C.c_double * max(len(self.dpow), 1))(*self.dpow)
        K = C.qcpd_cones(self.n_zero, self.n_nonneg, len(self.soc), soc, len(self.psd), psd,
                         self.n_exp, len(self.pow), pw, len(self.dpow), dp)
        return K, (soc, psd, pw, dp)


@dataclasses.dataclass
class Opts:
    tol: float = 1e-8
    max_iter: int = 0
    precond: int = C.QCPD_PRECOND_JACOBI
    graph_chunk: int = 128
    check_symmetry: int = 1
    engine: int = C.QCPD_ENGINE_AUTO
    solver: int = C.QCPD_SOLVER_LSQR
    # launch layout, fixed at create (0 = the library's choice)
    staged: int = C.QCPD_CHOICE_AUTO
    deep: int = C.QCPD_CHOICE_AUTO
    nnz_per_lane_F: int = 0
    nnz_per_lane_FT: int = 0
    lanes_x: int = 0
    lanes_y: int = 0
    loop_grid: int = 0
    persist_grid: int = 0
    equil_sweeps: int = 0

    def to_c(self) -> C.qcpd_opts:
        return C.qcpd_opts(self.tol, self.max_iter, self.precond, self.graph_chunk,
                           self.check_symmetry, self.engine, self.solver, self.staged,
                           self.deep, self.nnz_per_lane_F, self.nnz_per_lane_FT,
                           self.lanes_x, self.lanes_y,
                           self.loop_grid, self.persist_grid, self.equil_sweeps)


@dataclasses.dataclass
class Info:
    iters: int
    est_residual: float
    rel_residual: float
    flags: int
    ms_total: float

    @staticmethod
    def from_c(i: C.qcpd_info) -> "Info":
        return Info(i.iters, i.est_residual, i.rel_residual, i.flags, i.ms_total)


class Handle:
    """Owns a qcpd_handle* and keeps the tensors its shapes describe."""

    def __init__(self, ptr, n, m, nnzP, nnzA, device, stream):
        self.ptr = ptr
        self.n, self.m, self.nnzP, self.nnzA = n, m, nnzP, nnzA
        self.device = device
        self.stream = stream
        self.create_status = 0

    @property
    def N(self):
        return self.n + self.m + 1

    def close(self):
        if self.ptr:
            _lib().qcpd_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def qcpd_status_str(status: int) -> str:
    return _lib().qcpd_status_str(int(status)).decode()


def qcpd_opts_default() -> Opts:
    o = C.qcpd_opts()
    _lib().qcpd_opts_default(ctypes.byref(o))
    return Opts(**{name: getattr(o, name) for name, _ in C.qcpd_opts._fields_})


def _csr(rowptr, colind, val, nrows, ncols, name):
    nnz = int(colind.numel())
    return C.qcpd_csr(nrows, ncols, nnz, _ptr(rowptr, torch.int32, name + ".rowptr", nrows + 1),
                      _ptr(colind, torch.int32, name + ".colind"),
                      _ptr(val, torch.float64, name + ".val", nnz))


def qcpd_create(P: tuple, A: tuple, q, b, cones: Cones, x, y, s,
                opts: Optional[Opts] = None, stream: Optional[torch.cuda.Stream] = None,
                raise_on_warning: bool = False) -> Handle:
    """P, A: (rowptr int32, colind int32, val float64) GPU tensors; P is n x n full
    symmetric, A is m x n. Returns a Handle; raises QCPDError on errors."""
    n = int(q.numel())
    m = int(b.numel())
    Pc = _csr(*P, n, n, "P")
    Ac = _csr(*A, m, n, "A")
    K, keep = cones.to_c()
    o = (opts or qcpd_opts_default()).to_c()
    dev = q.device
    strm = stream if stream is not None else torch.cuda.current_stream(dev)
    h = ctypes.c_void_p()
    with torch.cuda.device(dev):
        st = _lib().qcpd_create(ctypes.byref(h), ctypes.byref(Pc), ctypes.byref(Ac),
                                _ptr(q, torch.float64, "q", n), _ptr(b, torch.float64, "b", m),
                                ctypes.byref(K), _ptr(x, torch.float64, "x", n),
                                _ptr(y, torch.float64, "y", m), _ptr(s, torch.float64, "s", m),
                                ctypes.byref(o), ctypes.c_void_p(strm.cuda_stream))
    if st < 0 or (raise_on_warning and st > 0):
        raise QCPDError(st, "qcpd_create")
    out = Handle(h, n, m, Pc.nnz, Ac.nnz, dev, strm)
    out.create_status = st
    return out


def qcpd_jvp(h: Handle, dP, dA, dq, db, dx=None, dy=None, ds=None):
    """Returns (dx, dy, ds, Info, status)."""
    f64 = dict(dtype=torch.float64, device=h.device)
    dx = torch.empty(h.n, **f64) if dx is None else dx
    dy = torch.empty(h.m, **f64) if dy is None else dy
    ds = torch.empty(h.m, **f64) if ds is None else ds
    info = C.qcpd_info()
    with torch.cuda.device(h.device):
        st = _lib().qcpd_jvp(h.ptr, _ptr(dP, torch.float64, "dP", h.nnzP),
                             _ptr(dA, torch.float64, "dA", h.nnzA),
                             _ptr(dq, torch.float64, "dq", h.n), _ptr(db, torch.float64, "db", h.m),
                             _ptr(dx, torch.float64, "dx", h.n), _ptr(dy, torch.float64, "dy", h.m),
                             _ptr(ds, torch.float64, "ds", h.m), ctypes.byref(info))
    if st < 0:
        raise QCPDError(st, "qcpd_jvp")
    return dx, dy, ds, Info.from_c(info), st


def qcpd_vjp(h: Handle, gx, gy, gs, dP=None, dA=None, dq=None, db=None):
    """Returns (dP, dA, dq, db, Info, status)."""
    f64 = dict(dtype=torch.float64, device=h.device)
    dP = torch.empty(h.nnzP, **f64) if dP is None else dP
    dA = torch.empty(h.nnzA, **f64) if dA is None else dA
    dq = torch.empty(h.n, **f64) if dq is None else dq
    db = torch.empty(h.m, **f64) if db is None else db
    info = C.qcpd_info()
    with torch.cuda.device(h.device):
        st = _lib().qcpd_vjp(h.ptr, _ptr(gx, torch.float64, "gx", h.n),
                             _ptr(gy, torch.float64, "gy", h.m), _ptr(gs, torch.float64, "gs", h.m),
                             _ptr(dP, torch.float64, "dP", h.nnzP),
                             _ptr(dA, torch.float64, "dA", h.nnzA),
                             _ptr(dq, torch.float64, "dq", h.n), _ptr(db, torch.float64, "db", h.m),
                             ctypes.byref(info))
    if st < 0:
        raise QCPDError(st, "qcpd_vjp")
    return dP, dA, dq, db, Info.from_c(info), st


def qcpd_set_opts(h: Handle, opts: Opts):
    o = opts.to_c()
    st = _lib().qcpd_set_opts(h.ptr, ctypes.byref(o))
    if st < 0:
        raise QCPDError(st, "qcpd_set_opts")


def qcpd_set_precond(h: Handle, d_col, d_row):
    """Two-sided scaling for QCPD_PRECOND_CUSTOM: the JVP solves with diag(d_row) F
    diag(d_col), the VJP with the transposed pair."""
    with torch.cuda.device(h.device):
        st = _lib().qcpd_set_precond(h.ptr, _ptr(d_col, torch.float64, "d_col", h.N),
                                     _ptr(d_row, torch.float64, "d_row", h.N))
    if st < 0:
        raise QCPDError(st, "qcpd_set_precond")


def qcpd_get_diagnostics(h: Handle):
    """Returns dict of new GPU tensors: jacobi_jvp, jacobi_vjp, equil_col, equil_row, jdiag."""
    f64 = dict(dtype=torch.float64, device=h.device)
    out = {k: torch.empty(h.N, **f64) for k in ("jacobi_jvp", "jacobi_vjp", "equil_col", "equil_row")}
    j = torch.empty(max(h.m, 1), **f64)
    with torch.cuda.device(h.device):
        st = _lib().qcpd_get_diagnostics(h.ptr, *[_ptr(out[k], torch.float64, k) for k in
                                                  ("jacobi_jvp", "jacobi_vjp", "equil_col", "equil_row")],
                                         _ptr(j, torch.float64, "jdiag"))
    if st < 0:
        raise QCPDError(st, "qcpd_get_diagnostics")
    out["jdiag"] = j[:h.m]
    return out


def qcpd_profile_kernels(h: Handle, reps: int = 50):
    """Average durations (ms) of the LSQR-iteration launches of the JVP: [the product with F,
    the product with F' (all its launches), its first launch alone, its second launch alone
    (0 when it has one)]."""
    out = (ctypes.c_float * 4)()
    with torch.cuda.device(h.device):
        st = _lib().qcpd_profile_kernels(h.ptr, int(reps), out)
    if st < 0:
        raise QCPDError(st, "qcpd_profile_kernels")
    return list(out)


@dataclasses.dataclass
class ResolveInfo:
    newton_iters: int
    lsqr_iters: int
    residual: float
    converged: bool


def qcpd_proj_dual(h: Handle, zy, out=None):
    """out = Pi_{K*}(zy) with the handle's cone spec (m entries)."""
    out = torch.empty(h.m, dtype=torch.float64, device=h.device) if out is None else out
    with torch.cuda.device(h.device):
        st = _lib().qcpd_proj_dual(h.ptr, _ptr(zy, torch.float64, "zy", h.m),
                                   _ptr(out, torch.float64, "out", h.m))
    if st < 0:
        raise QCPDError(st, "qcpd_proj_dual")
    return out


def qcpd_resolve(P: tuple, A: tuple, q, b, cones: Cones, x, y, s, tol: float = 1e-12,
                 max_newton: int = 20, opts: Optional[Opts] = None,
                 stream: Optional[torch.cuda.Stream] = None):
    """Newton refinement of (x, y, s) to a solution of the QCP (P, A, q, b, cones): the
    inputs are the starting point and are left as they are; returns (x, y, s, ResolveInfo,
    status) with new tensors."""
    n = int(q.numel())
    m = int(b.numel())
    Pc = _csr(*P, n, n, "P")
    Ac = _csr(*A, m, n, "A")
    K, keep = cones.to_c()
    o = (opts or qcpd_opts_default()).to_c()
    dev = q.device
    strm = stream if stream is not None else torch.cuda.current_stream(dev)
    xo, yo, so = x.detach().clone(), y.detach().clone(), s.detach().clone()
    info = C.qcpd_resolve_info()
    with torch.cuda.device(dev):
        st = _lib().qcpd_resolve(ctypes.byref(Pc), ctypes.byref(Ac),
                                 _ptr(q, torch.float64, "q", n), _ptr(b, torch.float64, "b", m),
                                 ctypes.byref(K), _ptr(xo, torch.float64, "x", n),
                                 _ptr(yo, torch.float64, "y", m), _ptr(so, torch.float64, "s", m),
                                 ctypes.byref(o), float(tol), int(max_newton), ctypes.byref(info),
                                 ctypes.c_void_p(strm.cuda_stream))
    if st < 0:
        raise QCPDError(st, "qcpd_resolve")
    return xo, yo, so, ResolveInfo(info.newton_iters, info.lsqr_iters, info.residual,
                                   bool(info.converged)), st


def qcpd_apply(h: Handle, v, transpose: bool = False, out=None):
    """out = F v (or F' v): the operator of the least-squares problems, unscaled."""
    out = torch.empty(h.N, dtype=torch.float64, device=h.device) if out is None else out
    with torch.cuda.device(h.device):
        st = _lib().qcpd_apply(h.ptr, int(bool(transpose)), _ptr(v, torch.float64, "v", h.N),
                               _ptr(out, torch.float64, "out", h.N))
    if st < 0:
        raise QCPDError(st, "qcpd_apply")
    return out


def qcpd_set_launch(h: Handle, grid_F: int = 0, grid_FT: int = 0):
    """Workgroup caps of the two LSQR-loop launches (0 = library default)."""
    with torch.cuda.device(h.device):
        st = _lib().qcpd_set_launch(h.ptr, int(grid_F), int(grid_FT))
    if st < 0:
        raise QCPDError(st, "qcpd_set_launch")


def qcpd_get_launch(h: Handle):
    """(grid_F, grid_FT, max_F, max_FT)."""
    out = (C.c_int32 * 4)()
    st = _lib().qcpd_get_launch(h.ptr, out)
    if st < 0:
        raise QCPDError(st, "qcpd_get_launch")
    return tuple(out)


def qcpd_get_layout(h: Handle) -> dict:
    """The launch layout chosen at create: staged, deep, psd_split, lanes_x, lanes_y,
    packed (the staged kernels' packed copies of P and A)."""
    out = (C.c_int32 * 6)()
    st = _lib().qcpd_get_layout(h.ptr, out)
    if st < 0:
        raise QCPDError(st, "qcpd_get_layout")
    return dict(zip(("staged", "deep", "psd_split", "lanes_x", "lanes_y", "packed"), tuple(out)))


def qcpd_destroy(h: Handle):
    h.close()
