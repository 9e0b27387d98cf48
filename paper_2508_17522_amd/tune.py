"""Autotuner for the launch shapes of the LSQR loops.

Single problem: the workgroup caps of the two loop launches (qcpd_set_launch) and the number
of LSQR iterations per captured graph (opts.graph_chunk). Batch: the lane schedule of its loop
kernels (entries per lane of a CSR row, opts.nnz_per_lane_F, fixed at create: each candidate
is a new handle) and the number of persistent workgroups (qcpd_batch_set_launch).

Each candidate is timed on the caller's own handle over a fixed number of LSQR iterations
(tolerance 0, so every candidate does the same work), best of `reps`. Results are cached in a
JSON file keyed by the device name and a shape bucket (powers of two of N and of the stored
entries), so a later handle of similar shape reuses the choice without timing.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Iterable, Optional, Tuple

import torch

from . import _capi as C
from .api import Handle, Opts, qcpd_get_launch, qcpd_jvp, qcpd_set_launch, qcpd_set_opts
from .batch import (BatchHandle, qcpd_batch_get_launch, qcpd_batch_jvp, qcpd_batch_set_launch,
                    qcpd_batch_set_opts)

CACHE_ENV = "QCPD_TUNE_CACHE"


def default_cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache",
                                                     "qcpd_tune.json")


def _bucket(v: int) -> int:
    return int(math.ceil(math.log2(max(int(v), 1))))


def shape_key(kind: str, device, N: int, nnz: int, extra: str = "") -> str:
    name = torch.cuda.get_device_name(device)
    return f"{kind}|{name}|N2^{_bucket(N)}|nnz2^{_bucket(nnz)}{extra}"


class TuneCache:
    def __init__(self, path: Optional[str] = None):
        self.path = path or default_cache_path()
        self.data: Dict[str, dict] = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.data = json.load(f)

    def get(self, key):
        return self.data.get(key)

    def put(self, key, value):
        self.data[key] = value
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def _probe_inputs(h: Handle, seed: int = 0):
    """A JVP input with a non-zero right-hand side (dq ~ N(0, 1), the rest zero)."""
    g = torch.Generator(device=h.device).manual_seed(seed)
    z = lambda k: torch.zeros(k, dtype=torch.float64, device=h.device)
    dq = torch.randn(h.n, generator=g, dtype=torch.float64, device=h.device)
    return z(h.nnzP), z(h.nnzA), dq, z(h.m)


def _time_handle(h: Handle, inputs, opts: Opts, reps: int) -> float:
    qcpd_set_opts(h, opts)
    best = math.inf
    for _ in range(reps):
        *_, info, _ = qcpd_jvp(h, *inputs)
        best = min(best, info.ms_total / max(info.iters, 1))
    return best


def default_candidates(max_F: int, max_FT: int) -> Iterable[Tuple[int, int, int]]:
    grids_F = sorted({min(max_F, g) for g in (128, 256, 512, 1024, 2048)})
    grids_T = sorted({min(max_FT, g) for g in (128, 256, 512, 1024, 2048)})
    for chunk in (16, 32, 64):
        for gF in grids_F:
            for gT in grids_T:
                yield gF, gT, chunk


def tune_handle(h: Handle, opts: Opts, *, iters: int = 200, reps: int = 2,
                cache: Optional[TuneCache] = None, force: bool = False,
                candidates: Optional[Iterable[Tuple[int, int, int]]] = None) -> dict:
    """Pick (grid_F, grid_FT, graph_chunk) for this handle and apply it. `opts` are the
    options the caller solves with (its preconditioner and engine); the returned dict holds
    the choice and the measured milliseconds per LSQR iteration."""
    key = shape_key("single", h.device, h.N, h.nnzP + 2 * h.nnzA, f"|prec{opts.precond}")
    if cache is not None and not force:
        hit = cache.get(key)
        if hit:
            qcpd_set_launch(h, hit["grid_F"], hit["grid_FT"])
            qcpd_set_opts(h, Opts(**{**opts.__dict__, "graph_chunk": hit["graph_chunk"]}))
            return dict(hit, cached=True)
    _, _, max_F, max_FT = qcpd_get_launch(h)
    inputs = _probe_inputs(h)
    results = []
    for gF, gT, chunk in (candidates or default_candidates(max_F, max_FT)):
        qcpd_set_launch(h, gF, gT)
        o = Opts(**{**opts.__dict__, "tol": 0.0, "max_iter": iters, "graph_chunk": chunk})
        results.append((_time_handle(h, inputs, o, reps), gF, gT, chunk))
    results.sort()
    ms, gF, gT, chunk = results[0]
    qcpd_set_launch(h, gF, gT)
    qcpd_set_opts(h, Opts(**{**opts.__dict__, "graph_chunk": chunk}))
    best = dict(grid_F=gF, grid_FT=gT, graph_chunk=chunk, ms_per_iter=ms,
                tried=len(results), worst_ms_per_iter=results[-1][0])
    if cache is not None:
        cache.put(key, best)
    return dict(best, cached=False)


def tune_batch(hb: BatchHandle, inputs, opts: Opts, *, iters: int = 100, reps: int = 2,
               cache: Optional[TuneCache] = None, force: bool = False,
               grids: Optional[Iterable[int]] = None) -> dict:
    """Pick the persistent grid of the batch kernel. `inputs` = (dP, dA, dq, db) of the batch
    (a JVP input); every candidate runs `iters` LSQR iterations per problem."""
    sN = sum(hb.n) + sum(hb.m) + hb.nprob
    key = shape_key("batch", hb.device, sN, sum(hb.nnzP) + 2 * sum(hb.nnzA),
                    f"|B2^{_bucket(hb.nprob)}")
    if cache is not None and not force:
        hit = cache.get(key)
        if hit:
            qcpd_batch_set_launch(hb, hit["grid"])
            return dict(hit, cached=True)
    _, dflt = qcpd_batch_get_launch(hb)
    if grids is None:
        ncu = torch.cuda.get_device_properties(hb.device).multi_processor_count
        grids = sorted({g for g in (ncu // 2, ncu, 2 * ncu, 3 * ncu, 4 * ncu, dflt, hb.nprob)
                        if 1 <= g <= hb.nprob})
    o = Opts(**{**opts.__dict__, "tol": 0.0, "max_iter": iters})
    qcpd_batch_set_opts(hb, o)
    results = []
    for g in grids:
        qcpd_batch_set_launch(hb, g)
        best = math.inf
        for _ in range(reps):
            *_, infos, _ = qcpd_batch_jvp(hb, *inputs)
            best = min(best, infos[0].ms_total)
        results.append((best, g))
    results.sort()
    ms, g = results[0]
    qcpd_batch_set_launch(hb, g)
    qcpd_batch_set_opts(hb, opts)
    out = dict(grid=g, ms=ms, default_grid=dflt,
               default_ms=next((t for t, gg in results if gg == dflt), None), tried=len(results))
    if cache is not None:
        cache.put(key, out)
    return dict(out, cached=False)


def tune_batch_lanes(make, inputs, opts: Opts, *, candidates: Iterable[int] = (8, 16, 32, 64),
                     iters: int = 100, reps: int = 2, cache: Optional[TuneCache] = None,
                     force: bool = False):
    """Pick the batch's entries per lane of a CSR row (opts.nnz_per_lane_F). `make(opts)`
    creates the batch handle for given options (the candidates differ at create); `inputs` =
    (dP, dA, dq, db) of a JVP. Every candidate runs `iters` LSQR iterations per problem
    (tolerance 0). Returns (handle created with the chosen options, those options, report);
    the other candidates' handles are closed."""
    best_h, report = None, None
    probe = make(opts)
    sN = sum(probe.n) + sum(probe.m) + probe.nprob
    key = shape_key("batch_lanes", probe.device, sN, sum(probe.nnzP) + 2 * sum(probe.nnzA),
                    f"|B2^{_bucket(probe.nprob)}|prec{opts.precond}")
    hit = cache.get(key) if (cache is not None and not force) else None
    if hit:
        chosen = Opts(**{**opts.__dict__, "nnz_per_lane_F": hit["nnz_per_lane"]})
        if hit["nnz_per_lane"] == opts.nnz_per_lane_F:
            return probe, chosen, dict(hit, cached=True)
        probe.close()
        return make(chosen), chosen, dict(hit, cached=True)
    probe.close()
    timing = Opts(**{**opts.__dict__, "tol": 0.0, "max_iter": iters})
    results = []
    for spl in candidates:
        o = Opts(**{**timing.__dict__, "nnz_per_lane_F": int(spl)})
        hb = make(o)
        best = math.inf
        for _ in range(reps):
            *_, infos, _ = qcpd_batch_jvp(hb, *inputs)
            best = min(best, infos[0].ms_total)
        hb.close()
        results.append((best, int(spl)))
    results.sort()
    ms, spl = results[0]
    chosen = Opts(**{**opts.__dict__, "nnz_per_lane_F": spl})
    report = dict(nnz_per_lane=spl, ms=ms, tried={str(s_): t for t, s_ in results})
    if cache is not None:
        cache.put(key, report)
    best_h = make(chosen)
    return best_h, chosen, dict(report, cached=False)
