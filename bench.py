"""Benchmark: JVP+VJP solves per second on one MI355X, FP64, LSQR relative residual 1e-8.

One step (one "solve") = create a handle at the solution (setup: copies, A', Px, cone
projections and Jacobian factors including the PSD eigendecompositions, scales) + one JVP +
one VJP, on the PSD/SOC-heavy workload n = 20000, m = 290000 (nonneg 15000, 2000 SOC(10),
200 PSD 50x50; A ~3M entries, P = BB' of rank 200), synthetic and seeded; --workload
mixed_qcp runs the n = 5000, m = 11000 mixed-cone workload instead. All inputs are resident
in HBM before the timed region.

Prints ONE JSON line. Also reports the LSQR iteration counts, the setup/JVP/VJP split, the
roofline position of the dominant kernel (algorithmic bytes per launch / its average launch
time, measured with HIP events on the library's stream) and the CPU oracle timed on a
bounded sample on this host.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large_psd_soc]
       python bench.py --workload batch [--batch-count 512]   (batched form, one launch)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "JVP+VJP solves/sec at 1e-8 rel. residual; LSQR iters & HBM GB/s vs plain"
HBM_PEAK_GBS = 8000.0


def _quads(indptr) -> int:
    import numpy as np
    return int((((np.diff(indptr) + 3) // 4) * 4).sum())


def kernel_bytes(q, which: str, packed: bool = False) -> float:
    """Algorithmic bytes of one launch of an LSQR-iteration kernel (JVP configuration):
    every CSR stream once (8 B value + 4 B column per entry, 4 B per row pointer; where the
    staged kernels read the packed copies of P and A, 8 B value + 2 B column per entry of rows
    padded to whole quads) and every vector it must read or write once."""
    n, m = q.n, q.m
    N = n + m + 1
    nnzP, nnzA = q.P.nnz, q.A.nnz
    if packed:
        pa = 10.0 * (_quads(q.P.indptr) + _quads(q.A.indptr))
    else:
        pa = 12.0 * (nnzP + nnzA)
    csr = pa + 12.0 * nnzA + 4.0 * (2 * n + m + 3)
    if which == "k_loop_F":
        # in, scale, J-input wy, q, b, out read+write, LSQR x and w read+write
        vec = 8.0 * (N + N + m + n + m + 2 * N + 4 * N)
        return csr + vec
    c = q.cones
    fac = 8.0 * (4 * len(c.soc) + sum(c.soc) + 9 * c.n_exp + sum(2 * k * k for k in c.psd))
    n_diag = c.n_zero + c.n_nonneg
    m_c = m - n_diag  # rows of non-diagonal cone blocks
    if which == "k_loop_FT":
        # in, c, b, out read+write, scale, jdiag of diagonal rows, wy write
        return csr + fac + 8.0 * (N + n + m + 2 * N + N + n_diag + m)
    if which == "k_loop_FT_rows":
        # the first of two launches: in, scale, c, b of the diagonal rows, out read+write of
        # the x rows, diagonal rows and tau, jdiag and wy of the diagonal rows, and the raw
        # cone rows written for the second launch
        return csr + 8.0 * (2 * N + n + n_diag + 2 * (n + n_diag + 1) + 2 * n_diag + m_c)
    if which == "k_loop_FT_cones":
        # the second launch: the cone factors, and per cone row its raw row, in, scale, b,
        # out read+write, wy write
        return fac + 8.0 * 7 * m_c
    raise ValueError(which)


def profiled_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed profiler counters of this workload
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), or None when there are none or the
    kernel's sources have changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_loop_{workload}.traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    h = hashlib.sha256()
    for src in t["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != t["sources_sha256"] or kernel not in t["kernels"]:
        return None
    return t["kernels"][kernel]["hbm_bytes_per_launch"]


def _oracle_rates(q, threads, budget_s):
    """Setup time and seconds per LSQR iteration of each direction of the oracle (numpy /
    scipy as it stands) with `threads` BLAS threads: a short run of each direction and a
    longer one sized to the budget; the difference of the two cancels the fixed costs
    (right-hand side, scales, first products)."""
    from threadpoolctl import threadpool_limits

    from oracle import derivative as D
    from oracle import embedding as E

    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        emb = E.Embedding(q)
        t_setup = time.perf_counter() - t0

        def run(direction, k):
            t0 = time.perf_counter()
            if direction == "jvp":
                D.jvp(q, q.dP, q.dA, q.dq, q.db, tol=1e-300, max_iter=k, emb=emb)
            else:
                D.vjp(q, q.gx, q.gy, q.gs, tol=1e-300, max_iter=k, emb=emb)
            return time.perf_counter() - t0

        rates, counts = {}, {}
        for direction in ("jvp", "vjp"):
            k0 = 2
            t_short = run(direction, k0)
            per = max(t_short / k0, 1e-9)
            k1 = int(min(20000, max(k0 + 8, 0.5 * budget_s / per)))
            t_long = run(direction, k1)
            rates[direction] = max(t_long - t_short, 1e-12) / (k1 - k0)
            counts[direction] = k1
    return t_setup, rates, counts


def cpu_baseline(q, iters_jvp, iters_vjp, budget_s=20.0):
    """The oracle on this host on a bounded sample, at one thread and with every core
    available to its BLAS: per-iteration times of both directions x the GPU's iteration
    counts, plus the oracle's setup at the solution. `value` is the faster of the two."""
    ncores = len(os.sched_getaffinity(0)) or 1
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():  # the host's share for this process
        ncores = max(1, min(ncores, int(os.environ["OMP_NUM_THREADS"])))
    out = {}
    for threads in (1, ncores):
        t_setup, rates, counts = _oracle_rates(q, threads, budget_s / 2)
        t_solve = t_setup + rates["jvp"] * iters_jvp + rates["vjp"] * iters_vjp
        out[threads] = dict(value=1.0 / t_solve, setup_s=t_setup, s_per_iter_jvp=rates["jvp"],
                            s_per_iter_vjp=rates["vjp"], sampled_iters=counts)
    best = max(out, key=lambda k: out[k]["value"])
    return {
        "value": out[best]["value"],
        "unit": "solves/s",
        "cores": best,
        "kind": "oracle",
        "sample": (f"oracle (numpy/scipy) setup at the solution + {out[best]['sampled_iters']['jvp']} "
                   f"LSQR iterations of the JVP and {out[best]['sampled_iters']['vjp']} of the VJP on "
                   f"the same workload with {best} BLAS thread(s) (scipy's sparse products use one); "
                   f"per-iteration time x the GPU's iteration counts ({iters_jvp} JVP + "
                   f"{iters_vjp} VJP); {ncores} cores available"),
        "nproc": ncores,
        "one_thread": {k: out[1][k] for k in ("value", "setup_s", "s_per_iter_jvp", "s_per_iter_vjp")},
        "all_cores": {k: out[ncores][k] for k in ("value", "setup_s", "s_per_iter_jvp", "s_per_iter_vjp")},
    }


def run_batch(args):
    """Batched form: `count` uneven problems (n ~ U{20..400}, m ~ U{1.5n..3n}) per launch.
    One step = batch create + batch JVP + batch VJP over all of them; the value counts every
    problem's JVP+VJP as one solve. vs_plain times the single-problem Jacobi path over the
    first `plain` problems."""
    import numpy as np
    import torch

    import paper_2508_17522_amd as Q
    import qcpgen
    from qcpgen.torch_io import batch_create_args, batch_to_device, cones_of, to_device

    count = args.batch_count
    print(f"[bench] generating {count} batch problems", file=sys.stderr, flush=True)
    qs = [qcpgen.batch_member(i) for i in range(count)]
    bt = batch_to_device(qs)
    prec = {"equil": Q.QCPD_PRECOND_EQUIL, "jacobi": Q.QCPD_PRECOND_JACOBI,
            "none": Q.QCPD_PRECOND_NONE}[args.precond]
    opts = Q.Opts(tol=args.tol, precond=prec)
    tuned = None
    if not args.no_tune:
        # the autotuner's lane schedule for this batch (entries per lane of a CSR row), chosen
        # before the timed region on 100 LSQR iterations per candidate
        from paper_2508_17522_amd import tune as T
        hb0, opts, tuned = T.tune_batch_lanes(
            lambda o: Q.qcpd_batch_create(*batch_create_args(bt), opts=o),
            (bt["dP"], bt["dA"], bt["dq"], bt["db"]), opts, cache=T.TuneCache())
        hb0.close()
        print(f"[bench] tuned batch lanes: {tuned}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    def step(record):
        t0 = time.perf_counter()
        hb = Q.qcpd_batch_create(*batch_create_args(bt), opts=opts)
        t1 = time.perf_counter()
        _, _, _, ij, sj = Q.qcpd_batch_jvp(hb, bt["dP"], bt["dA"], bt["dq"], bt["db"])
        t2 = time.perf_counter()
        _, _, _, _, iv, sv = Q.qcpd_batch_vjp(hb, bt["gx"], bt["gy"], bt["gs"])
        t3 = time.perf_counter()
        hb.close()
        if record is not None:
            record.append(dict(setup=t1 - t0, jvp=t2 - t1, vjp=t3 - t2, ij=ij, iv=iv, sj=sj, sv=sv))

    for i in range(args.warmup):
        step(None)
        print(f"[bench] warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    rec = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(rec)
        print(f"[bench] step {i + 1}/{args.steps}: jvp {rec[-1]['jvp']:.3f}s vjp "
              f"{rec[-1]['vjp']:.3f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    value = count * args.steps / elapsed
    bad = [i for i, r in enumerate(rec)
           if r["sj"] != 0 or r["sv"] != 0
           or max(x.rel_residual for x in r["ij"] + r["iv"]) > args.tol]
    if bad:
        print(f"[bench] WARNING: {len(bad)} timed step(s) did not converge: {bad}",
              file=sys.stderr, flush=True)
    last = rec[-1]
    it_j = [i.iters for i in last["ij"]]
    it_v = [i.iters for i in last["iv"]]
    # roofline of the segmented LSQR loop over the whole JVP: algorithmic bytes of every
    # problem's LSQR iterations / the JVP's duration (HIP events on the library's stream)
    per_iter = [kernel_bytes(q, "k_loop_F") + kernel_bytes(q, "k_loop_FT") for q in qs]
    t_launch = last["ij"][0].ms_total * 1e-3
    nbytes = float(sum(b * k for b, k in zip(per_iter, it_j)))
    achieved = nbytes / t_launch / 1e9
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch_member x{count} (uneven, one launch)",
                   "sum_N": int(sum(q.n + q.m + 1 for q in qs)),
                   "sum_nnz_P": int(sum(q.P.nnz for q in qs)),
                   "sum_nnz_A": int(sum(q.A.nnz for q in qs)), "tol": args.tol,
                   "precond": args.precond,
                   "nnz_per_lane": opts.nnz_per_lane_F or 32, "tuned": tuned},
        "lsqr_iters": {"jvp_median": float(np.median(it_j)), "jvp_max": int(max(it_j)),
                       "vjp_median": float(np.median(it_v)), "vjp_max": int(max(it_v))},
        "max_rel_residual": {"jvp": max(i.rel_residual for i in last["ij"]),
                             "vjp": max(i.rel_residual for i in last["iv"])},
        "status": {"jvp": last["sj"], "vjp": last["sv"]},
        "all_steps_converged": not bad,
        "split_ms": {k: round(1e3 * float(np.median([r[k] for r in rec])), 3)
                     for k in ("setup", "jvp", "vjp")},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                     "kernel": "k_seg_F + k_seg_FT (every iteration of the JVP)",
                     "jvp_us": round(t_launch * 1e6, 3), "bytes": int(nbytes)},
    }
    if args.batch_plain > 0:
        k = min(args.batch_plain, count)
        print(f"[bench] plain single-problem Jacobi LSQR over {k} problems", file=sys.stderr,
              flush=True)
        o2 = Q.Opts(tol=args.tol, precond=Q.QCPD_PRECOND_JACOBI)
        tens = [to_device(q) for q in qs[:k]]
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for q, t in zip(qs[:k], tens):
            h = Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones_of(q), t["x"], t["y"],
                              t["s"], opts=o2)
            Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"])
            Q.qcpd_vjp(h, t["gx"], t["gy"], t["gs"])
            h.close()
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        line["vs_plain"] = {"precond": "jacobi", "path": "one problem per call",
                            "problems": k, "value": round(k / tp, 3), "unit": "solves/s",
                            "speedup": round(value / (k / tp), 3)}
        if args.precond != "jacobi":  # the same preconditioner, one problem per call
            o3 = Q.Opts(tol=args.tol, precond=prec)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            for q, t in zip(qs[:k], tens):
                h = Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones_of(q), t["x"], t["y"],
                                  t["s"], opts=o3)
                Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"])
                Q.qcpd_vjp(h, t["gx"], t["gy"], t["gs"])
                h.close()
            torch.cuda.synchronize()
            ts = time.perf_counter() - ts
            line["vs_single_same_precond"] = {"precond": args.precond, "path": "one problem per call",
                                              "problems": k, "value": round(k / ts, 3),
                                              "unit": "solves/s", "speedup": round(value / (k / ts), 3)}
    print(json.dumps(line), flush=True)


def copy_bandwidth(mib: int = 1024, launches: int = 20) -> float:
    """GB/s (bytes read + written) of a plain device-to-device copy of `mib` MiB, timed with
    HIP events after one untimed copy: the bandwidth a plain stream reaches on this GPU."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(launches):
        dst.copy_(src)
    t1.record()
    t1.synchronize()
    us = t0.elapsed_time(t1) * 1e3 / launches
    del src, dst
    return 2 * n * 8 / us / 1e3


def run_copy_calibration(mib: int):
    """A plain device-to-device copy of known size (the reference for scaling the HBM byte
    counters of a profiler run): reads and writes `mib` MiB per launch, 20 launches."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(20):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    gbs = copy_bandwidth(mib)  # 21 more copies of the same size, timed
    print(json.dumps({"copy_calibration": {"bytes_read_per_launch": n * 8,
                                           "bytes_written_per_launch": n * 8, "launches": 20,
                                           "GBps_read_plus_write": round(gbs, 1)}}),
          flush=True)


LAYOUT_FIELDS = ("staged", "deep", "nnz_per_lane_F", "nnz_per_lane_FT", "lanes_x", "lanes_y",
                 "loop_grid")


def layout_opts(args) -> dict:
    """--layout FIELD=VALUE pairs as Opts keyword arguments."""
    out = {}
    for item in args.layout:
        k, _, v = item.partition("=")
        if k not in LAYOUT_FIELDS:
            raise SystemExit(f"bench.py: unknown layout field {k!r} (one of {LAYOUT_FIELDS})")
        out[k] = int(v)
    return out


# single kernels of an LSQR iteration (the symbols a profiler shows) -> their byte model
BYTES_OF = {"k_loop_F": "k_loop_F", "k_loop_F_xs": "k_loop_F", "k_loop_FT": "k_loop_FT",
            "k_loop_FT_xs": "k_loop_FT_rows", "k_loop_FT rows form": "k_loop_FT_rows",
            "k_loop_FT_cones": "k_loop_FT_cones"}


def launch_bytes(q, name, layout) -> float:
    """The byte model of a launch; the staged kernels read the packed copies of P and A."""
    return kernel_bytes(q, BYTES_OF[name], packed=name.endswith("_xs"))


def launch_times(ms, layout) -> dict:
    """The launches of one iteration by kernel, from qcpd_profile_kernels' four durations."""
    staged = layout["staged"] == 1
    out = {"k_loop_F_xs" if staged else "k_loop_F": ms[0]}
    if ms[3] > 0.0:
        out["k_loop_FT_xs" if staged else "k_loop_FT rows form"] = ms[2]
        out["k_loop_FT_cones"] = ms[3]
    else:
        out["k_loop_FT_xs" if staged else "k_loop_FT"] = ms[1]
    return out


def run_kernels_only(args):
    """Setup of the workload, then each LSQR-loop kernel launched back to back (for counter
    runs of a profiler: a few hundred dispatches instead of a whole solve)."""
    import torch

    import paper_2508_17522_amd as Q
    import qcpgen
    from qcpgen.torch_io import cones_of, to_device
    q = qcpgen.make(args.workload, 0)
    t = to_device(q)
    prec = {"equil": Q.QCPD_PRECOND_EQUIL, "jacobi": Q.QCPD_PRECOND_JACOBI,
            "none": Q.QCPD_PRECOND_NONE}[args.precond]
    h = Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones_of(q), t["x"], t["y"], t["s"],
                      opts=Q.Opts(tol=args.tol, precond=prec, **layout_opts(args)))
    layout = Q.qcpd_get_layout(h)
    ms = Q.qcpd_profile_kernels(h, reps=args.kernels_only)
    h.close()
    torch.cuda.synchronize()
    us = {k: v * 1e3 for k, v in launch_times(ms, layout).items()}
    nb = {k: launch_bytes(q, k, layout) for k in us}
    gbs = {k: nb[k] / us[k] / 1e3 for k in us}
    print(json.dumps({"kernels_only": {"workload": q.name, "reps": args.kernels_only,
                                       "layout": layout,
                                       "avg_launch_us": us, "bytes_per_launch": nb,
                                       "achieved_GBps": gbs,
                                       "frac_of_hbm_peak": {k: gbs[k] / HBM_PEAK_GBS for k in us}}}),
          flush=True)


def run_resolve(args):
    """The forward solve by refinement on the workload: theta moved by a seeded step of
    relative size --resolve-step along random directions on the patterns, the old solution as
    the starting point, Newton steps to --resolve-tol (qcpd_resolve). Timed with the GPU
    synchronised on both sides; the oracle's dense re-solve of the same data is timed beside
    it when n + m <= 4 000 (it factors the dense reduced KKT matrix at every step)."""
    import numpy as np
    import torch

    import paper_2508_17522_amd as Q
    import qcpgen
    from qcpgen.torch_io import cones_of, to_device
    q = qcpgen.make(args.workload, 0)
    rng = np.random.default_rng([7, q.n, q.m])
    h = args.resolve_step
    dP = qcpgen.symmetric_on_pattern(rng, q.P, 1.0)
    dA, dq, db = (rng.standard_normal(k) for k in (q.A.nnz, q.n, q.m))
    P1 = q.P.copy()
    P1.data = q.P.data + h * np.abs(q.P.data).mean() * dP
    A1 = q.A.copy()
    A1.data = q.A.data + h * np.abs(q.A.data).mean() * dA
    q1 = q.q + h * np.abs(q.q).mean() * dq
    b1 = q.b + h * np.abs(q.b).mean() * db
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")
    t = to_device(q)
    Pd = (t["P"][0], t["P"][1], f(P1.data))
    Ad = (t["A"][0], t["A"][1], f(A1.data))
    prec = {"equil": Q.QCPD_PRECOND_EQUIL, "jacobi": Q.QCPD_PRECOND_JACOBI,
            "none": Q.QCPD_PRECOND_NONE}[args.precond]
    opts = Q.Opts(tol=args.tol, precond=prec, **layout_opts(args))
    runs = []
    for rep in range(args.steps + args.warmup):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, y, s, info, st = Q.qcpd_resolve(Pd, Ad, f(q1), f(b1), cones_of(q), t["x"], t["y"],
                                           t["s"], tol=args.resolve_tol, opts=opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(f"[bench] resolve {rep + 1}: {dt:.3f} s, {info.newton_iters} steps, "
              f"{info.lsqr_iters} LSQR iterations, residual {info.residual:.2e}",
              file=sys.stderr, flush=True)
        if rep >= args.warmup:
            runs.append(dt)
    moved = float(np.linalg.norm(x.cpu().numpy() - q.x) / max(np.linalg.norm(q.x), 1e-300))
    out = {"resolve": {"workload": q.name, "theta_step": h, "tol": args.resolve_tol,
                       "lsqr_tol": args.tol, "precond": args.precond,
                       "seconds_median": float(np.median(runs)), "runs": len(runs),
                       "newton_iters": info.newton_iters, "lsqr_iters": info.lsqr_iters,
                       "residual": info.residual, "status": st,
                       "relative_change_of_x": moved}}
    if q.n + q.m <= 4000 and not args.no_cpu_baseline:
        from oracle import derivative as D
        from oracle import embedding as E
        qp = E.with_data(q, h * np.abs(q.P.data).mean() * dP, h * np.abs(q.A.data).mean() * dA,
                         h * np.abs(q.q).mean() * dq, h * np.abs(q.b).mean() * db)
        t0 = time.perf_counter()
        xr, yr, sr, res = D.newton_resolve(qp, q.x, q.y - q.s)
        out["resolve"]["cpu_baseline"] = {
            "seconds": time.perf_counter() - t0, "kind": "oracle", "residual": res,
            "sample": "the oracle's dense semismooth Newton re-solve of the same data",
            "max_rel_diff_x": float(np.linalg.norm(x.cpu().numpy() - xr) / np.linalg.norm(xr))}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large_psd_soc")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precond", default="equil", choices=["equil", "jacobi", "none"])
    ap.add_argument("--solver", default="lsqr", choices=["lsqr", "lsmr"],
                    help="the Krylov method of the derivative solves (LSMR: the paper's)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain Jacobi-preconditioned LSQR comparison")
    ap.add_argument("--plain-max-iter", type=int, default=100000,
                    help="iteration cap of each direction of the plain Jacobi comparison")
    ap.add_argument("--engine", default="auto", choices=["auto", "graph", "persistent"])
    ap.add_argument("--batch-count", type=int, default=512,
                    help="problems per launch for --workload batch")
    ap.add_argument("--batch-plain", type=int, default=64,
                    help="problems timed on the single-problem path for --workload batch")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (profiler byte-counter reference)")
    ap.add_argument("--resolve", action="store_true",
                    help="time the forward solve by refinement after a step in theta")
    ap.add_argument("--resolve-step", type=float, default=1e-3,
                    help="relative size of the step in theta for --resolve")
    ap.add_argument("--resolve-tol", type=float, default=1e-10,
                    help="stopping tolerance of the refinement for --resolve")
    ap.add_argument("--kernels-only", type=int, default=0, metavar="REPS",
                    help="only set up the workload and launch each loop kernel REPS times")
    ap.add_argument("--no-tune", action="store_true",
                    help="batch workload: keep the library's default lane schedule")
    ap.add_argument("--layout", action="append", default=[], metavar="FIELD=VALUE",
                    help="a launch-layout option of the library (staged, deep, nnz_per_lane_F, "
                         "nnz_per_lane_FT, lanes_x, lanes_y, loop_grid), for tuning runs; "
                         "repeatable")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (--gpus 1); the derivative of one QCP is not "
              "split across GPUs.", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        run_copy_calibration(args.copy_calibration)
        return
    if args.kernels_only:
        run_kernels_only(args)
        return
    if args.resolve:
        run_resolve(args)
        return
    if args.workload == "batch":
        run_batch(args)
        return

    import numpy as np
    import torch

    import paper_2508_17522_amd as Q
    import qcpgen
    from qcpgen.torch_io import cones_of, to_device

    q = qcpgen.make(args.workload, 0)
    dev = "cuda:0"
    t = to_device(q, dev)
    cones = cones_of(q)
    PREC = {"equil": Q.QCPD_PRECOND_EQUIL, "jacobi": Q.QCPD_PRECOND_JACOBI,
            "none": Q.QCPD_PRECOND_NONE}
    prec = PREC[args.precond]
    eng = {"auto": Q.QCPD_ENGINE_AUTO, "graph": Q.QCPD_ENGINE_GRAPH,
           "persistent": Q.QCPD_ENGINE_PERSISTENT}[args.engine]
    solver = {"lsqr": Q.QCPD_SOLVER_LSQR, "lsmr": Q.QCPD_SOLVER_LSMR}[args.solver]
    opts = Q.Opts(tol=args.tol, precond=prec, engine=eng, solver=solver, **layout_opts(args))
    outs = dict(dx=torch.empty(q.n, dtype=torch.float64, device=dev),
                dy=torch.empty(q.m, dtype=torch.float64, device=dev),
                ds=torch.empty(q.m, dtype=torch.float64, device=dev),
                dP=torch.empty(q.P.nnz, dtype=torch.float64, device=dev),
                dA=torch.empty(q.A.nnz, dtype=torch.float64, device=dev),
                dq=torch.empty(q.n, dtype=torch.float64, device=dev),
                db=torch.empty(q.m, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()

    def step(record, o=None):
        t0 = time.perf_counter()
        h = Q.qcpd_create(t["P"], t["A"], t["q"], t["b"], cones, t["x"], t["y"], t["s"],
                          opts=o or opts)
        t1 = time.perf_counter()
        _, _, _, ij, sj = Q.qcpd_jvp(h, t["dP"], t["dA"], t["dq"], t["db"],
                                    outs["dx"], outs["dy"], outs["ds"])
        t2 = time.perf_counter()
        _, _, _, _, iv, sv = Q.qcpd_vjp(h, t["gx"], t["gy"], t["gs"], outs["dP"], outs["dA"],
                                       outs["dq"], outs["db"])
        t3 = time.perf_counter()
        if record is not None:
            record.append(dict(setup=t1 - t0, jvp=t2 - t1, vjp=t3 - t2, ij=ij, iv=iv, sj=sj, sv=sv))
        return h

    for i in range(args.warmup):
        step(None).close()
        print(f"[bench] warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    rec = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        h = step(rec)
        h.close()
        print(f"[bench] step {i + 1}/{args.steps}: jvp {rec[-1]['ij'].iters} it "
              f"{rec[-1]['jvp']:.2f}s, vjp {rec[-1]['iv'].iters} it {rec[-1]['vjp']:.2f}s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    value = args.steps / elapsed
    # a timed step counts only if both solves converged: status OK and the recomputed
    # relative residual at or below the tolerance
    bad = [i for i, r in enumerate(rec)
           if r["sj"] != 0 or r["sv"] != 0 or not (r["ij"].rel_residual <= args.tol)
           or not (r["iv"].rel_residual <= args.tol)]
    if bad:
        print(f"[bench] WARNING: {len(bad)} timed step(s) did not converge: {bad}",
              file=sys.stderr, flush=True)

    # roofline of the dominant kernel: average launch duration measured with HIP events
    h = step(None)
    layout = Q.qcpd_get_layout(h)
    ms = Q.qcpd_profile_kernels(h, reps=200)
    h.close()
    iters_total = rec[-1]["ij"].iters + rec[-1]["iv"].iters
    times = launch_times(ms, layout)
    dom_name = max(times, key=times.get)
    nbytes = launch_bytes(q, dom_name, layout)
    achieved = nbytes / (times[dom_name] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": profiled_traffic(q.name, dom_name),
                "kernel": dom_name, "avg_launch_us": round(times[dom_name] * 1e3, 3),
                "bytes_per_launch": int(nbytes),
                "all_kernels_us": {k: round(v * 1e3, 3) for k, v in times.items()},
                "frac_by_kernel": {k: round(launch_bytes(q, k, layout) / (v * 1e-3) / 1e9
                                            / HBM_PEAK_GBS, 4) for k, v in times.items()},
                "us_per_iteration": round((ms[0] + ms[1]) * 1e3, 3)}
    copy_gbs = copy_bandwidth()
    roofline["measured_copy_GBps"] = round(copy_gbs, 1)
    roofline["frac_of_measured_copy"] = round(achieved / copy_gbs, 4)

    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": q.name, "n": q.n, "m": q.m, "nnz_P": int(q.P.nnz),
                   "nnz_A": int(q.A.nnz), "tol": args.tol, "precond": args.precond,
                   "engine": args.engine, "solver": args.solver,
                   "cones": {"zero": q.cones.n_zero, "nonneg": q.cones.n_nonneg,
                             "soc": len(q.cones.soc), "psd": len(q.cones.psd),
                             "exp": q.cones.n_exp}},
        "lsqr_iters": {"jvp": rec[-1]["ij"].iters, "vjp": rec[-1]["iv"].iters},
        "rel_residual": {"jvp": max(r["ij"].rel_residual for r in rec),
                         "vjp": max(r["iv"].rel_residual for r in rec)},
        "all_steps_converged": not bad,
        "split_ms": {k: round(1e3 * float(np.median([r[k] for r in rec])), 3)
                     for k in ("setup", "jvp", "vjp")},
        "us_per_lsqr_iter": round(1e6 * float(np.median([r["jvp"] + r["vjp"] for r in rec]))
                                  / max(iters_total, 1), 3),
        "roofline": roofline,
    }
    if not args.no_plain and args.precond != "jacobi":
        # plain Jacobi-preconditioned LSQR on the same GPU, same stopping tolerance
        print("[bench] plain Jacobi LSQR for comparison", file=sys.stderr, flush=True)
        plain = []
        o2 = Q.Opts(tol=args.tol, precond=Q.QCPD_PRECOND_JACOBI, engine=eng,
                    max_iter=args.plain_max_iter)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        step(plain, o2).close()
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        line["vs_plain"] = {"precond": "jacobi", "value": round(1.0 / tp, 4),
                            "unit": "solves/s", "speedup": round(value * tp, 3),
                            "lsqr_iters": {"jvp": plain[0]["ij"].iters, "vjp": plain[0]["iv"].iters},
                            "rel_residual": {"jvp": plain[0]["ij"].rel_residual,
                                             "vjp": plain[0]["iv"].rel_residual},
                            "max_iter": args.plain_max_iter,
                            "converged": plain[0]["sj"] == 0 and plain[0]["sv"] == 0}
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(q, rec[-1]["ij"].iters, rec[-1]["iv"].iters)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
