#!/usr/bin/env python3
"""Benchmark of the SpMV + Krylov hot path on one MI355X.

Default workload ("spmv_set"): the 48 held-out synthetic FP64 matrices (four
families x twelve sizes, n = 1e4 .. 2e6).  One step runs the method's whole
SpMV path on every matrix: ingest (copy + validate), GPU features, cascaded
prediction, format conversion when the prediction asks for it, then 200
products with the predicted kernel (the paper times configurations as the
mean of 200 runs).  The next matrix is prepared on a second stream while the
current one's products run; the sequential step is reported beside it.
value = algorithmic bytes of all those products / step time, in GB/s.

Untimed, the same run measures every configuration on every matrix (warm,
200 products each) to report predicted vs exhaustive-best vs default CSR-vector,
times the predicted / best / default kernels cold (cache flushed) on the
matrices whose product moves >= 512 MB, and times the CPU oracle on one
product per matrix.

Other workloads (--workload): cg_lap2d (CG, 64x64 Laplacian), cg_async (async
CG on 3D Poisson 128^3 and a 2^20-row power-law graph Laplacian),
gmres_mixed (mixed vs FP64 GMRES(30), convection-diffusion 1024^2), serve
(request loop), select_latency (host vs device-resident cascade).  Each
prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SpMV HBM GB/s (predicted vs best vs CSR); CG/GMRES solves/s + p99 @1e-10"
HBM_PEAK_GBS = 8000.0
LARGE_BYTES = 512 * 2 ** 20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class KernelLedger:
    """Event-timed batches of SpMV launches inside the timed steps, per device
    kernel symbol (HIP events recorded by the library on the launch stream)."""

    def __init__(self):
        self.k = {}

    def add(self, name, launches, us_per_launch, bytes_per_launch):
        e = self.k.setdefault(name, [0, 0.0, 0.0])
        e[0] += launches
        e[1] += launches * us_per_launch
        e[2] += launches * bytes_per_launch

    def summary(self, name):
        n, us, by = self.k[name]
        return dict(launches=n, avg_us=us / n, achieved_GBs=by / (us * 1e3))

    def dominant(self):
        """Kernel with the largest total time."""
        return max(self.k, key=lambda name: self.k[name][1])


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def flush_cache(buf):
    buf.fill_(1.0)   # 1 GiB streaming write evicts the 256 MB last-level cache


def geomean(v):
    v = [x for x in v if x > 0 and math.isfinite(x)]
    return math.exp(sum(math.log(x) for x in v) / len(v)) if v else float("nan")


def traffic_for(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, if
    it was taken for this kernel (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        return d.get(kernel)
    except Exception:
        return None


# ---------------------------------------------------------------------------
def bench_spmv_set(args):
    import torch

    import paper_2411_10143_amd as ck
    from synth import workloads as W

    torch.cuda.set_device(0)
    specs = W.spmv_set_specs(max_n=args.max_n)
    if args.only:
        specs = [sp for sp in specs if sp[0].startswith(args.only + "_")]
        if not specs:
            raise SystemExit(f"--only {args.only}: no such member of the SpMV set")
    mats, dev = [], []
    t0 = time.time()
    for i, spec in enumerate(specs):
        A = W.spmv_set_matrix(spec)
        mats.append(A)
        dev.append(dict(rp=torch.from_numpy(A.rp).cuda(), col=torch.from_numpy(A.col).cuda(),
                        val=torch.from_numpy(A.val).cuda(),
                        x=torch.from_numpy(np.random.default_rng(spec[4]).uniform(-1, 1, A.ncols)).cuda(),
                        y=torch.zeros(A.n, dtype=torch.float64, device="cuda")))
        log(f"[gen {i + 1}/{len(specs)}] {A.name} n={A.n} nnz={A.nnz} ({time.time() - t0:.0f}s)")
    nbytes = [A.nnz * 12 + 4 * (A.n + 1) + 8 * A.ncols + 8 * A.n for A in mats]
    ledger = KernelLedger()
    R = args.reps

    # ---- exhaustive table (warm, every configuration) -----------------------
    T = np.full((len(mats), ck.NUM_CONFIGS), np.inf)
    default_id, ablation_ids = [], []
    for m, (A, d) in enumerate(zip(mats, dev)):
        Mx = ck.Matrix(d["rp"], d["col"], d["val"], A.ncols)
        default_id.append(ck.config_id(ck.default_config(Mx.handle)))
        if args.no_table:
            Mx.close()
            continue
        ablation_ids.append(single_stage_picks(ck, ck.spmv_features(Mx.handle),
                                               ck.default_config(Mx.handle)))
        for cid in range(ck.NUM_CONFIGS):
            cfg = ck.config_from_id(cid)
            try:
                ck.spmv_convert(Mx.handle, cfg)
            except ck.CkError as e:
                if e.status != ck.CK_E_UNSUPPORTED:
                    raise
                continue
            T[m, cid] = ck.time_spmv(Mx.handle, cfg, d["x"], d["y"], warmup=10, reps=R)
        Mx.close()
        log(f"[table {m + 1}/{len(mats)}] {A.name} best={ck.CONFIG_NAMES[int(np.argmin(T[m]))]}"
            f" {T[m].min():.2f}us default={T[m, default_id[-1]]:.2f}us")

    # ---- timed steps: ingest -> features -> select -> convert -> R products ---
    # every device block of the step's handles from torch's caching allocator
    # (the binding's default), or from the library's own cache.  Pipelined
    # (the default): a worker thread prepares matrix m + 1 (ingest, features,
    # cascade, conversion) on a second stream while matrix m's products run
    # on the main stream -- the paper's overlap of preprocessing with
    # execution, across the batch.  Sequential: the same calls one after the
    # other on the main stream.
    from concurrent.futures import ThreadPoolExecutor
    alloc = None if args.allocator == "library" else "torch"
    phase_ms = dict(ingest=0.0, features=0.0, select=0.0, convert=0.0, products=0.0,
                    release=0.0, exposed_prep=0.0)
    side = torch.cuda.Stream()          # default priority
    pool = ThreadPoolExecutor(max_workers=1)

    def prepare(m, stream):
        A, d = mats[m], dev[m]
        clk = time.perf_counter
        t0 = clk()
        Mx = ck.Matrix(d["rp"], d["col"], d["val"], A.ncols, stream=stream, allocator=alloc)
        t1 = clk()
        F = ck.spmv_features(Mx.handle, stream=stream, symmetry=False)   # the cascade's inputs
        t2 = clk()
        cfg = ck.spmv_select(F)
        t3 = clk()
        try:
            ck.spmv_convert(Mx.handle, cfg, stream=stream)
        except ck.CkError as e:
            if e.status != ck.CK_E_UNSUPPORTED:
                raise
            cfg = ck.default_config(Mx.handle)   # refused conversion: keep the default
        if stream is not None:
            stream.synchronize()             # all the products read is complete
        t4 = clk()
        return Mx, cfg, (t0, t1, t2, t3, t4)

    def prepare_side(m):
        with torch.cuda.stream(side):
            return prepare(m, side)

    def one_step(record, pipelined=True):
        picks, spmv_us = [], 0.0
        clk = time.perf_counter
        fut = pool.submit(prepare_side, 0) if pipelined else None
        for m, (A, d) in enumerate(zip(mats, dev)):
            tw = clk()
            if pipelined:
                Mx, cfg, tp = fut.result()
                if m + 1 < len(mats):
                    fut = pool.submit(prepare_side, m + 1)
            else:
                Mx, cfg, tp = prepare(m, None)
            t4 = clk()
            us = ck.time_spmv(Mx.handle, cfg, d["x"], d["y"], warmup=0, reps=R)
            t5 = clk()
            spmv_us += us * R
            if record:
                ledger.add(ck.kernel_name(cfg), R, us, nbytes[m])
            picks.append(ck.config_id(cfg))
            Mx.close()
            t6 = clk()
            if record:   # host wall time per phase (the preparation overlaps when pipelined)
                for k, a, b in (("ingest", tp[0], tp[1]), ("features", tp[1], tp[2]),
                                ("select", tp[2], tp[3]), ("convert", tp[3], tp[4]),
                                ("products", t4, t5), ("release", t5, t6),
                                ("exposed_prep", tw, t4)):
                    phase_ms[k] += (b - a) * 1e3
        return picks, spmv_us

    for _ in range(args.warmup):
        one_step(False)
    torch.cuda.synchronize()
    step_times, spmv_totals, picks = [], [], None
    for s in range(args.steps):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        picks, spmv_us = one_step(True)
        torch.cuda.synchronize()
        step_times.append(time.perf_counter() - ts)
        spmv_totals.append(spmv_us)
        log(f"[step {s + 1}/{args.steps}] {step_times[-1] * 1e3:.1f} ms")
    # the same step without the overlap, for comparison (not the bench value)
    seq_times = []
    for s in range(max(2, args.steps // 4)):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        one_step(False, pipelined=False)
        torch.cuda.synchronize()
        seq_times.append(time.perf_counter() - ts)
    pool.shutdown()
    bytes_step = R * sum(nbytes)
    value = bytes_step * len(step_times) / sum(step_times) / 1e9

    # the kernel with the largest total time inside the timed steps
    dominant = ledger.dominant()
    ks = ledger.summary(dominant)

    # ---- cold products on the large matrices ---------------------------------
    cold = []
    flushbuf = torch.empty(2 ** 27, dtype=torch.float64, device="cuda")
    for m, (A, d) in enumerate(zip(mats, dev)):
        if nbytes[m] < LARGE_BYTES or args.no_table:
            continue
        Mx = ck.Matrix(d["rp"], d["col"], d["val"], A.ncols)
        row = dict(matrix=A.name, MB=round(nbytes[m] / 1e6, 1))
        for label, cid in (("predicted", picks[m]), ("best", int(np.argmin(T[m]))),
                           ("default", default_id[m])):
            cfg = ck.config_from_id(cid)
            ck.spmv_convert(Mx.handle, cfg)
            ts = []
            for _ in range(5):
                flush_cache(flushbuf)
                ts.append(ck.time_spmv(Mx.handle, cfg, d["x"], d["y"], warmup=0, reps=1))
            us = float(np.median(ts))
            row[label] = dict(config=ck.CONFIG_NAMES[cid], us=round(us, 2),
                              GBs=round(nbytes[m] / (us * 1e3), 1),
                              frac=round(nbytes[m] / (us * 1e3) / HBM_PEAK_GBS, 3))
        cold.append(row)
        Mx.close()
    del flushbuf

    # ---- achievable copy bandwidth (same box) ---------------------------------
    a = torch.empty(2 ** 28, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    copy_gbs = 10 * 2 * a.numel() * 8 / (e0.elapsed_time(e1) * 1e6)
    del a, b

    # ---- CPU oracle baseline ---------------------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        xs = [d["x"].cpu().numpy() for d in dev]

        def passes_for(seconds, parallel):
            # whole passes over the set (one product per matrix each)
            passes = 0
            tc = time.perf_counter()
            while passes == 0 or (time.perf_counter() - tc < seconds and passes < 400):
                for A, x in zip(mats, xs):
                    oracle.spmv(A, x, parallel=parallel)
                passes += 1
            return passes, time.perf_counter() - tc

        pa, dta = passes_for(8.0, True)
        p1, dt1 = passes_for(8.0, False)
        threads = oracle.threads(parallel=True)
        cpu = dict(value=round(pa * sum(nbytes) / dta / 1e9, 3), unit="GB/s", cores=threads,
                   kind="oracle",
                   sample=f"{pa} passes of one FP64 product per matrix of the "
                          f"{len(mats)}-matrix set ({sum(nbytes) / 1e9:.2f} GB algorithmic per "
                          f"pass), plain C with OpenMP over rows on {threads} threads, "
                          f"{dta:.1f} s; host has {os.cpu_count()} logical CPUs ({_cpu_model()})",
                   single_core=dict(value=round(p1 * sum(nbytes) / dt1 / 1e9, 3), unit="GB/s",
                                    cores=1, sample=f"{p1} passes, {dt1:.1f} s"))

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * sum(step_times) / len(step_times), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"spmv_set_{len(mats)}: banded/power-law/block-diagonal/"
                               f"uniform-random FP64, n 1e4-2e6, int32 CSR; per matrix ingest + "
                               f"GPU features + cascade + conversion + {R} products, the next "
                               f"matrix prepared on a second stream during the products",
                   "matrices": len(mats), "products_per_matrix": R,
                   "algorithmic_GB_per_step": round(bytes_step / 1e9, 3)},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(ks["achieved_GBs"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ks["achieved_GBs"] / HBM_PEAK_GBS, 4),
                     "avg_us": round(ks["avg_us"], 3), "launches": ks["launches"],
                     "traffic": traffic_for(dominant)},
        "cpu_baseline": cpu,
        "spmv": {
            "kernel_GBs_in_steps": round(bytes_step / (np.mean(spmv_totals) * 1e3), 1),
            "step_phase_ms": {k: round(v / len(step_times), 2) for k, v in phase_ms.items()},
            "sequential_step": {"GBs": round(R * sum(nbytes) * len(seq_times) / sum(seq_times) / 1e9, 1),
                                "ms_per_step": round(1e3 * sum(seq_times) / len(seq_times), 3),
                                "steps": len(seq_times)},
            "copy_GBs": round(copy_gbs, 1),
            "kernels_in_steps": {k: dict(launches=v[0], avg_us=round(v[1] / v[0], 3))
                                 for k, v in sorted(ledger.k.items())},
        },
    }
    if not args.no_table:
        # predicted vs exhaustive-best vs default, all from the warm table
        best = T.min(axis=1)
        t_pred = np.array([T[m, p] for m, p in enumerate(picks)])
        t_def = np.array([T[m, default_id[m]] for m in range(len(mats))])
        ratio = t_pred / best
        agg = lambda t: float(sum(nbytes) / (np.sum(t) * 1e3))   # GB/s over the set
        # single-stage predictors (only one part of the configuration predicted,
        # the rest at the default) against the full cascade
        abl = {}
        for key in ("format_only", "algorithm_only", "lanes_only"):
            t = np.array([T[m, ablation_ids[m][key]] if math.isfinite(T[m, ablation_ids[m][key]])
                          else T[m, default_id[m]] for m in range(len(mats))])
            abl[key] = dict(GBs=round(agg(t), 1), geomean_t_over_t_best=round(geomean(t / best), 4))
        abl["cascade"] = dict(GBs=round(agg(t_pred), 1),
                              geomean_t_over_t_best=round(geomean(ratio), 4))
        # the known-inputs start tree (no pass over the entries) against the
        # default rule, both among the configurations that need no copy
        t_start = np.array([T[m, ck.config_id(ck.start_config(A.n, A.ncols, A.nnz)[0])]
                            for m, A in enumerate(mats)])
        best9 = T[:, :9].min(axis=1)
        known = dict(GBs=round(agg(t_start), 1), best_no_copy_GBs=round(agg(best9), 1),
                     geomean_t_over_t_best_no_copy=round(geomean(t_start / best9), 4),
                     default_geomean_t_over_t_best_no_copy=round(geomean(t_def / best9), 4))
        out["spmv"].update({
            "single_stage_ablation": abl, "known_start": known,
            "predicted_GBs": round(agg(t_pred), 1), "best_GBs": round(agg(best), 1),
            "default_csr_vector_GBs": round(agg(t_def), 1),
            "geomean_t_pred_over_t_best": round(geomean(ratio), 4),
            "geomean_t_default_over_t_best": round(geomean(t_def / best), 4),
            "picked_best": int(np.sum(ratio <= 1.0)), "within_10pct": int(np.sum(ratio <= 1.10)),
            "of": len(mats), "cold_large": cold})
    if not args.no_solvers:
        try:
            out["solvers"] = solver_summary(args)
        except Exception as e:            # the SpMV line stands on its own
            log(f"[solvers] failed: {e!r}")
            out["solvers"] = {"error": repr(e)}
    if args.table and not args.no_table:
        rows = []
        for m, A in enumerate(mats):
            rows.append(dict(matrix=A.name, n=A.n, nnz=A.nnz, MB=round(nbytes[m] / 1e6, 2),
                             times_us=[None if not math.isfinite(v) else round(v, 3) for v in T[m]],
                             predicted=ck.CONFIG_NAMES[picks[m]],
                             best=ck.CONFIG_NAMES[int(np.argmin(T[m]))],
                             default=ck.CONFIG_NAMES[default_id[m]]))
        with open(args.table, "w") as f:
            json.dump(rows, f, indent=1)
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# Solver workloads.  The solve is timed from the call to the result on the
# host, with the matrix resident; `roofline` reports the effective bandwidth
# of the iteration (algorithmic bytes of all iterations / solve time).

def _solve_json(args, value, unit, ms_per_step, workload, extra, roof, cpu, dtype="f64"):
    out = {"metric": METRIC, "value": round(value, 3), "unit": unit, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic", "config": dict(workload=workload, **extra.pop("config", {})),
           "roofline": roof, "cpu_baseline": cpu}
    out.update(extra)
    print(json.dumps(out), flush=True)


def _cg_iter_bytes(A, s=8):
    # fused CG iteration: SpMV (+p.Ap) then x,r update (+r.r) then p update
    return A.nnz * (s + 4) + 4 * (A.n + 1) + 2 * s * A.n + 6 * s * A.n + 3 * s * A.n


def _gmres_iter_bytes(A, m=30, s=8):
    # SpMV, three Gram-Schmidt passes over j+1 basis columns (average m/2 + 1),
    # normalisation; per-cycle residual and update terms amortised over m
    spmv = A.nnz * (s + 4) + 4 * (A.n + 1) + 2 * s * A.n
    cols = m / 2.0 + 1.0
    return spmv + s * A.n * (3 * cols + 2 + 2 + 1 + 2 + 2) + (8 * A.n * (4 + m)) / m


def _upload(A):
    import torch
    return (torch.from_numpy(A.rp).cuda(), torch.from_numpy(A.col).cuda(),
            torch.from_numpy(A.val).cuda())


def _rhs(ck, Mx, xs):
    import torch
    dx = torch.from_numpy(xs).cuda()
    b = torch.zeros_like(dx)
    ck.spmv_apply(Mx.handle, dx, b)
    return b


def bench_cg_lap2d(args):
    import torch

    import paper_2411_10143_amd as ck
    from synth import workloads as W
    A, xs = W.lap2d_64()
    Mx = ck.Matrix.from_csr(A)
    b = _rhs(ck, Mx, xs)
    per_step = 20
    lat, iters = [], []
    for s in range(args.warmup + args.steps):
        for _ in range(per_step):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = ck.cg_solve(Mx.handle, b, x, tol=1e-10)
            dt = time.perf_counter() - t
            assert r["status"] == ck.CK_OK and r["true_relres"] <= 1e-10, r
            if s >= args.warmup:
                lat.append(dt)
                iters.append(r["iterations"])
    total = sum(lat)
    eff = float(np.mean(iters)) * _cg_iter_bytes(A) / (total / len(lat)) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        bh = b.cpu().numpy()
        tc = time.perf_counter()
        n = 0
        while time.perf_counter() - tc < 10.0:
            oracle.cg(A, bh, tol=1e-10)
            n += 1
        dt = time.perf_counter() - tc
        cpu = dict(value=round(n / dt, 2), unit="solves/s", cores=1, kind="oracle",
                   sample=f"{n} complete oracle CG solves of the same system")
    _solve_json(args, len(lat) / total, "solves/s", 1e3 * total / args.steps,
                "cg_lap2d_64: FP64 CG, 2D 5-point Laplacian 64x64 (n=4096), tol 1e-10; "
                "the library's default path for n <= 4096: the whole solve in one "
                "single-workgroup launch (CSR-vector product, one lane per row, the "
                "matrix held in registers)",
                {"latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                                "p99": round(1e3 * float(np.percentile(lat, 99)), 3)},
                 "iterations": int(np.median(iters)), "solves": len(lat)},
                {"bound": "hbm", "kernel": "cg_wg<4> (single-workgroup CG)",
                 "achieved": round(eff, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(eff / HBM_PEAK_GBS, 5), "traffic": None,
                 "note": "n=4096: the whole system sits in one CU's registers and LDS; "
                         "latency-bound, not an HBM roofline claim"}, cpu)


def single_stage_picks(ck, F, default):
    """Configuration ids of the three single-stage predictors: each evaluates
    one stage's tree alone and keeps the default for the other parts."""
    f = ck.eval_stage(F, 0)
    a = ck.eval_stage(F, 1)
    lg = ck.eval_stage(F, 2)
    fmt_cfg = default if f == ck.CK_FMT_CSR else ck.Config(f, 0, 0, 0)
    alg_cfg = ck.Config(ck.CK_FMT_CSR, a, default.lanes if a == ck.CK_ALG_VECTOR else 0, 0)
    lanes_cfg = ck.Config(ck.CK_FMT_CSR, ck.CK_ALG_VECTOR, 1 << lg, 0)
    return {"format_only": ck.config_id(fmt_cfg), "algorithm_only": ck.config_id(alg_cfg),
            "lanes_only": ck.config_id(lanes_cfg)}


def _best_fixed_config(ck, Mx, A):
    import torch
    x = torch.ones(A.ncols, dtype=torch.float64, device="cuda")
    y = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    best, tb = None, math.inf
    for cid in range(ck.NUM_CONFIGS):
        cfg = ck.config_from_id(cid)
        try:
            ck.spmv_convert(Mx.handle, cfg)
        except ck.CkError:
            continue
        t = ck.time_spmv(Mx.handle, cfg, x, y, warmup=5, reps=50)
        if t < tb:
            best, tb = cid, t
    return best, tb


def bench_cg_async(args):
    import torch

    import paper_2411_10143_amd as ck
    from synth import workloads as W
    problems = [("poisson3d_128", *W.poisson3d_128()),
                ("graph_laplacian_2^20", *W.graph_laplacian_1m())]
    rows, tot_time, tot_solves, tot_bytes = [], 0.0, 0, 0.0
    for name, A, xs in problems:
        log(f"[cg_async] {name} n={A.n} nnz={A.nnz}")
        rp, col, val = _upload(A)
        probe = ck.Matrix(rp, col, val)
        b = _rhs(ck, probe, xs)
        best_id, _ = _best_fixed_config(ck, probe, A)
        probe.close()
        res = {"async": [], "async_overhead_aware": [], "async_known_start": [],
               "sequential": [], "default": [], "known_start": [], "best_fixed": []}
        for s in range(args.warmup + args.steps):
            for mode in res:
                Mx = ck.Matrix(rp, col, val)        # fresh handle: nothing cached
                kw = {}
                if mode == "async":
                    kw["async_"] = ck.CK_EXEC_ASYNC
                elif mode == "async_overhead_aware":
                    kw["async_"] = ck.CK_EXEC_ASYNC
                    kw["overhead_aware"] = True
                elif mode == "async_known_start":
                    kw["async_"] = ck.CK_EXEC_ASYNC
                    kw["known_start"] = True
                elif mode == "known_start":
                    kw["known_start"] = True
                elif mode == "sequential":
                    kw["async_"] = ck.CK_EXEC_SEQUENTIAL
                elif mode == "best_fixed":
                    kw["config"] = ck.config_from_id(best_id)
                    ck.spmv_convert(Mx.handle, kw["config"])
                x = torch.zeros_like(b)
                torch.cuda.synchronize()
                t = time.perf_counter()
                r = ck.cg_solve(Mx.handle, b, x, tol=1e-10, **kw)
                dt = time.perf_counter() - t
                assert r["status"] == ck.CK_OK, (name, mode, r)
                if s >= args.warmup:
                    r["wall_s"] = dt
                    if mode == "async":
                        r["forward_error"] = float(np.linalg.norm(x.cpu().numpy() - xs) /
                                                   np.linalg.norm(xs))
                    res[mode].append(r)
                Mx.close()
        a = res["async"]
        t_async = sum(r["wall_s"] for r in a)
        tot_time += t_async
        tot_solves += len(a)
        tot_bytes += sum(r["iterations"] for r in a) * _cg_iter_bytes(A)
        rows.append({"problem": name, "n": A.n, "nnz": A.nnz,
                     "async_solves_per_s": round(len(a) / t_async, 3),
                     "async_overhead_aware_solves_per_s": round(len(res["async_overhead_aware"]) / sum(r["wall_s"] for r in res["async_overhead_aware"]), 3),
                     "overhead_gate": {k: res["async_overhead_aware"][-1][k] for k in ("conversion_gated", "est_remaining_iters", "switch_iter")},
                     "async_known_start_solves_per_s": round(len(res["async_known_start"]) / sum(r["wall_s"] for r in res["async_known_start"]), 3),
                     "known_start_solves_per_s": round(len(res["known_start"]) / sum(r["wall_s"] for r in res["known_start"]), 3),
                     "known_start_config": ck.CONFIG_NAMES[ck.config_id(ck.start_config(A.n, A.ncols, A.nnz)[0])],
                     "sequential_solves_per_s": round(len(res["sequential"]) / sum(r["wall_s"] for r in res["sequential"]), 3),
                     "sequential_prep_us": round(sum(res["sequential"][-1][k] for k in ("t_features_us", "t_infer_us", "t_convert_us")), 1),
                     "default_solves_per_s": round(len(res["default"]) / sum(r["wall_s"] for r in res["default"]), 3),
                     "best_fixed_solves_per_s": round(len(res["best_fixed"]) / sum(r["wall_s"] for r in res["best_fixed"]), 3),
                     "best_fixed_config": ck.CONFIG_NAMES[best_id],
                     "iterations": a[-1]["iterations"], "switch_iter": a[-1]["switch_iter"],
                     "final_config": ck.CONFIG_NAMES[a[-1]["final_config"]],
                     "t_features_us": round(a[-1]["t_features_us"], 1),
                     "t_infer_us": round(a[-1]["t_infer_us"], 2),
                     "t_convert_us": round(a[-1]["t_convert_us"], 1),
                     "true_relres": a[-1]["true_relres"],
                     "forward_error": a[-1]["forward_error"],
                     "latency_ms": {"p50": round(1e3 * float(np.percentile([r["wall_s"] for r in a], 50)), 3),
                                    "p99": round(1e3 * float(np.percentile([r["wall_s"] for r in a], 99)), 3)}})
        del rp, col, val, b
    eff = tot_bytes / tot_time / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        A, xs = problems[0][1], problems[0][2]
        bh = oracle.spmv(A, xs)
        k = 20
        tc = time.perf_counter()
        oracle.cg(A, bh, tol=1e-30, maxit=k)
        dt = (time.perf_counter() - tc) / k
        it = rows[0]["iterations"]
        cpu = dict(value=round(1.0 / (dt * it), 5), unit="solves/s", cores=1, kind="oracle",
                   sample=f"{k} oracle CG iterations on poisson3d_128 ({dt * 1e3:.1f} ms each), "
                          f"scaled to the {it} iterations of a full solve")
    _solve_json(args, tot_solves / tot_time, "solves/s", 1e3 * tot_time / args.steps,
                "cg_async: async FP64 CG, tol 1e-10, on 3D Poisson 128^3 (n=2,097,152) and a "
                "Chung-Lu power-law graph Laplacian + 1e-2 I (n=2^20, mean degree 16)",
                {"problems": rows},
                {"bound": "hbm", "kernel": "cg_iteration (fused SpMV + 2 vector kernels)",
                 "achieved": round(eff, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(eff / HBM_PEAK_GBS, 4), "traffic": None}, cpu)


def bench_gmres_mixed(args):
    import torch

    import paper_2411_10143_amd as ck
    from synth import workloads as W
    A, xs = W.convdiff_1024(args.grid)
    log(f"[gmres_mixed] n={A.n} nnz={A.nnz}")
    Mx = ck.Matrix.from_csr(A, keep_fp32=True)
    b = _rhs(ck, Mx, xs)
    # the method's configuration for this matrix, predicted once and kept (as
    # the request loop's prediction cache does); both precisions use it
    cfg = ck.spmv_select(ck.spmv_features(Mx.handle))
    try:
        ck.spmv_convert(Mx.handle, cfg)
    except ck.CkError as e:
        if e.status != ck.CK_E_UNSUPPORTED:
            raise
        cfg = ck.default_config(Mx.handle)
    log(f"[gmres_mixed] predicted configuration {ck.CONFIG_NAMES[ck.config_id(cfg)]}")
    res = {"mixed": [], "fp64": []}
    for s in range(args.warmup + args.steps):
        for mode in res:
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = ck.gmres_solve(Mx.handle, b, x, tol=1e-10, restart=30, max_iter=200000,
                               precision=ck.CK_PREC_MIXED if mode == "mixed" else ck.CK_PREC_FP64,
                               config=cfg)
            dt = time.perf_counter() - t
            assert r["status"] == ck.CK_OK, (mode, r)
            log(f"[gmres_mixed] {mode} {dt:.3f}s it={r['iterations']} relres={r['true_relres']:.2e}")
            if s >= args.warmup:
                xh = x.cpu().numpy()
                r["wall_s"] = dt
                r["forward_error"] = float(np.linalg.norm(xh - xs) / np.linalg.norm(xs))
                r["x"] = xh
                res[mode].append(r)
    tm = sum(r["wall_s"] for r in res["mixed"])
    t64 = sum(r["wall_s"] for r in res["fp64"])
    mixed_sps, fp64_sps = len(res["mixed"]) / tm, len(res["fp64"]) / t64
    rm, r64 = res["mixed"][-1], res["fp64"][-1]
    eff = rm["iterations"] * _gmres_iter_bytes(A, 30, 4) / (tm / len(res["mixed"])) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        bh = b.cpu().numpy()
        k = 60
        tc = time.perf_counter()
        oracle.gmres(A, bh, m=30, tol=1e-30, maxit=k)
        dt = (time.perf_counter() - tc) / k
        cpu = dict(value=round(1.0 / (dt * r64["iterations"]), 6), unit="solves/s", cores=1,
                   kind="oracle",
                   sample=f"{k} oracle FP64 GMRES(30) iterations ({dt * 1e3:.1f} ms each), scaled "
                          f"to the {r64['iterations']} iterations of the GPU FP64 solve")
    keep = ("iterations", "outer_steps", "true_relres", "forward_error")
    _solve_json(args, mixed_sps, "solves/s", 1e3 * (tm + t64) / args.steps,
                f"gmres_mixed: GMRES(30), 2D convection-diffusion {args.grid}^2 upwind, "
                "Peclet 10, tol 1e-10; mixed FP32 inner / FP64 refinement vs plain FP64; "
                f"predicted SpMV configuration {ck.CONFIG_NAMES[ck.config_id(cfg)]}",
                {"mixed": {**{k: rm[k] for k in keep}, "solves_per_s": round(mixed_sps, 4)},
                 "fp64": {**{k: r64[k] for k in keep}, "solves_per_s": round(fp64_sps, 4)},
                 "mixed_vs_fp64_rel_diff": float(np.linalg.norm(rm["x"] - r64["x"]) /
                                                 np.linalg.norm(r64["x"])),
                 "mixed_speedup": round(mixed_sps / fp64_sps, 3)},
                {"bound": "hbm", "kernel": "mixed gmres_iteration (SpMV + CGS2 passes)",
                 "achieved": round(eff, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(eff / HBM_PEAK_GBS, 4), "traffic": None}, cpu, dtype="f32+f64")


def bench_serve(args):
    import paper_2411_10143_amd as ck
    from paper_2411_10143_amd.serving import ServingWorkload, latency_summary, poisson_arrivals
    from synth import workloads as W
    t0 = time.time()
    pool = W.serving_pool()
    log(f"[serve] pool of {len(pool)} matrices generated in {time.time() - t0:.0f}s; "
        f"n from {min(A.n for A, _ in pool)} to {max(A.n for A, _ in pool)}")
    Wl = ServingWorkload(pool, args.requests, tol=args.tol, precision=ck.CK_PREC_MIXED,
                         budget_bytes=64 << 30, max_slots=256, chunk_iters=args.chunk_iters,
                         small_n=args.small_n, large_workers=args.large_workers)
    log(f"[serve] {args.requests} requests prepared")
    # closed loop: capacity C (also warms the prediction cache and residency)
    prog = lambda m: log(f"[serve] {m}")
    cap = latency_summary(Wl.run(progress=prog))
    log(f"[serve] closed loop: {cap['solves_per_s']:.1f} solves/s")
    rate = args.rate if args.rate else 0.8 * cap["solves_per_s"]
    runs = []
    for s in range(args.steps):
        done = Wl.run(arrivals_s=poisson_arrivals(args.requests, rate, seed=5001 + s),
                      progress=prog)
        runs.append((latency_summary(done), done))
        log(f"[serve] open loop {s + 1}: p50 {runs[-1][0]['p50_ms']:.2f} ms "
            f"p99 {runs[-1][0]['p99_ms']:.2f} ms")
    summ, done = runs[-1]
    # every result's FP64 true residual, as the library recomputed it at exit
    worst = max(float(c["true_relres"]) for c in done)
    st = Wl.stats()
    Wl.close()
    mean_sps = float(np.mean([r[0]["solves_per_s"] for r in runs]))
    _solve_json(args, mean_sps, "solves/s",
                1e3 * float(np.mean([r[0]["makespan_s"] for r in runs])),
                f"serve: {args.requests} requests, Poisson arrivals at "
                f"{f'{rate:g}/s' if args.rate else '0.8x closed-loop capacity'}, 64-matrix pool (n log-uniform 1e3-1e6), CG if symmetric else "
                f"GMRES(30), mixed FP32/FP64, tol {args.tol:g}, batched slots for n <= {args.small_n}, "
                f"{args.chunk_iters} iterations per batched launch, "
                f"{args.large_workers} large-system workers",
                {"latency_ms": {"p50": round(summ["p50_ms"], 3), "p99": round(summ["p99_ms"], 3),
                                "mean": round(summ["mean_ms"], 3)},
                 "closed_loop_solves_per_s": round(cap["solves_per_s"], 3),
                 "arrival_rate_per_s": round(rate, 3),
                 "batched_fraction": round(summ["batched"] / summ["solves"], 3),
                 "ok": summ["ok"], "worst_true_relres": worst, "server_stats": st},
                {"bound": "hbm", "kernel": "batched_chunk + solver kernels", "achieved": None,
                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None, "traffic": None},
                None, dtype="f32+f64")


def bench_select_latency(args):
    """Prediction latency on the serving pool's 64 matrices (n 1e3-1e6),
    resident handle, cold prediction: host cascade (GPU feature pass, read
    back the accumulators, derive and walk the trees on the host) against the
    device-resident cascade (feature pass, derivation and walk on the GPU,
    read back the 8-int decision); both end with the decision on the host."""
    import torch

    import paper_2411_10143_amd as ck
    from synth import workloads as W
    pool = W.serving_pool()
    out = torch.zeros(8, dtype=torch.int32, device="cuda")
    rows = []
    for A, _sym in pool:
        Mx = ck.Matrix.from_csr(A)
        ck.select_device(Mx.handle, out)        # uploads the model once; keeps the scratch
        torch.cuda.synchronize()
        th, td, te = [], [], []
        for _ in range(args.steps + args.warmup):
            t0 = time.perf_counter()
            F = ck.spmv_features(Mx.handle, symmetry=False)
            cfg = ck.spmv_select(F)
            t1 = time.perf_counter()
            ck.select_device(Mx.handle, out)
            t2 = time.perf_counter()
            dev = out.cpu().tolist()
            t3 = time.perf_counter()
            assert dev[7] == ck.config_id(cfg), (A.name, dev, cfg)
            th.append(t1 - t0)
            td.append(t3 - t1)
            te.append(t2 - t1)
        Mx.close()
        k = args.warmup
        rows.append(dict(matrix=A.name, n=A.n, nnz=A.nnz, config=ck.CONFIG_NAMES[dev[7]],
                         host_us=round(1e6 * float(np.median(th[k:])), 1),
                         device_us=round(1e6 * float(np.median(td[k:])), 1),
                         device_enqueue_us=round(1e6 * float(np.median(te[k:])), 1)))
        log(f"[select] {A.name} n={A.n} host {rows[-1]['host_us']} us device "
            f"{rows[-1]['device_us']} us")
    h = np.array([r["host_us"] for r in rows])
    d = np.array([r["device_us"] for r in rows])
    small = np.array([r["n"] <= 32768 for r in rows])
    _solve_json(args, float(np.median(h / d)), "x (host / device prediction latency, median)",
                float(np.sum(h) + np.sum(d)) / 1e3,
                "select_latency: cold cascade prediction on the 64-matrix serving pool, "
                "host cascade vs device-resident cascade, decision read back on the host",
                {"median_host_us": float(np.median(h)), "median_device_us": float(np.median(d)),
                 "median_host_us_n_le_32768": float(np.median(h[small])),
                 "median_device_us_n_le_32768": float(np.median(d[small])),
                 "matrices": rows},
                {"bound": "hbm", "kernel": "feature pass + cascade_from_ints", "achieved": None,
                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None, "traffic": None}, None)


def _timed_solves(ck, fn, Mx, b, count, warmup=1, **kw):
    """Wall time of `count` solves from the call to the result on the host
    (the matrix resident), after `warmup` untimed ones; the last x and result."""
    import torch
    lat, r, x = [], None, None
    for i in range(warmup + count):
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn(Mx.handle, b, x, **kw)
        dt = time.perf_counter() - t
        assert r["status"] == ck.CK_OK, r
        if i >= warmup:
            lat.append(dt)
    return lat, r, x


def _lat(lat):
    return {"solves_per_s": round(len(lat) / sum(lat), 3),
            "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3), "solves": len(lat)}


def solver_summary(args):
    """The metric's solver half in the default run: CG on the 64x64 Laplacian
    (default path and the default CSR-vector kernel), async CG and mixed vs
    FP64 CG on the 3D Poisson and graph Laplacian systems, mixed vs FP64
    GMRES(30) on convection-diffusion 1024^2, and a shortened request-loop
    trace at tol 1e-10.  Each result's true residual is checked against the
    oracle's (all-core build)."""
    import torch

    import oracle
    import paper_2411_10143_amd as ck
    from paper_2411_10143_amd.serving import ServingWorkload, latency_summary, poisson_arrivals
    from synth import workloads as W
    out = {}
    fe = lambda x, xs: float(np.linalg.norm(x.cpu().numpy() - xs) / np.linalg.norm(xs))

    # -- CG, 2D Laplacian 64^2 ------------------------------------------------
    A, xs = W.lap2d_64()
    Mx = ck.Matrix.from_csr(A)
    b = _rhs(ck, Mx, xs)
    lat, r, x = _timed_solves(ck, ck.cg_solve, Mx, b, 100, 5, tol=1e-10)
    assert oracle.relres(A, b.cpu().numpy(), x.cpu().numpy()) <= 1e-10
    row = {"default_path": {**_lat(lat), "iterations": r["iterations"],
                            "kernel": "cg_wg<4>: whole solve in one workgroup, one lane per row, matrix in registers"}}
    cfg = ck.default_config(Mx.handle)
    lat, r, x = _timed_solves(ck, ck.cg_solve, Mx, b, 100, 5, tol=1e-10, config=cfg)
    assert oracle.relres(A, b.cpu().numpy(), x.cpu().numpy()) <= 1e-10
    row["default_csr_vector"] = {**_lat(lat), "iterations": r["iterations"],
                                 "kernel": f"batched_chunk, {ck.CONFIG_NAMES[ck.config_id(cfg)]} "
                                           "product, whole solve in one launch"}
    if not args.no_cpu_baseline:
        bh = b.cpu().numpy()
        for par in (True, False):
            n, tc = 0, time.perf_counter()
            while n < 5 or time.perf_counter() - tc < 3.0:
                oracle.cg(A, bh, tol=1e-10, parallel=par)
                n += 1
            dt = time.perf_counter() - tc
            row["cpu_oracle_all_cores" if par else "cpu_oracle_one_core"] = {
                "solves_per_s": round(n / dt, 2), "cores": oracle.threads(par),
                "sample": f"{n} complete oracle CG solves"}
    out["cg_lap2d_64"] = row
    Mx.close()
    log("[solvers] cg_lap2d_64 done")

    # -- CG on 3D Poisson 128^3 and the 2^20 graph Laplacian --------------------
    rows = {}
    for name, (A, xs) in (("poisson3d_128", W.poisson3d_128()),
                          ("graph_laplacian_2^20", W.graph_laplacian_1m())):
        Mx = ck.Matrix.from_csr(A, keep_fp32=True)
        b = _rhs(ck, Mx, xs)
        bh = b.cpu().numpy()
        cnt = 5 if A.n <= 2_200_000 and name.startswith("poisson") else 3
        lat, ra, x = _timed_solves(ck, ck.cg_solve, Mx, b, cnt, 1, tol=1e-10,
                                   async_=ck.CK_EXEC_ASYNC)
        rr = oracle.relres(A, bh, x.cpu().numpy(), parallel=True)
        assert rr <= 1e-10, (name, rr)
        row = {"n": A.n, "nnz": A.nnz,
               "async": {**_lat(lat), "iterations": ra["iterations"],
                         "switch_iter": ra["switch_iter"],
                         "final_config": ck.CONFIG_NAMES[ra["final_config"]],
                         "oracle_true_relres": rr, "forward_error": fe(x, xs)}}
        # mixed vs FP64 on the configuration the cascade predicts, kept fixed
        cfg = ck.spmv_select(ck.spmv_features(Mx.handle))
        try:
            ck.spmv_convert(Mx.handle, cfg)
        except ck.CkError as e:
            if e.status != ck.CK_E_UNSUPPORTED:
                raise
            cfg = ck.default_config(Mx.handle)
        for prec, key in ((ck.CK_PREC_FP64, "fp64"), (ck.CK_PREC_MIXED, "mixed")):
            lat, r, x = _timed_solves(ck, ck.cg_solve, Mx, b, 2 if cnt == 3 else 4, 1,
                                      tol=1e-10, precision=prec, config=cfg)
            rr = oracle.relres(A, bh, x.cpu().numpy(), parallel=True)
            assert rr <= 1e-10, (name, key, rr)
            row[key] = {**_lat(lat), "iterations": r["iterations"],
                        "outer_steps": r["outer_steps"], "oracle_true_relres": rr,
                        "forward_error": fe(x, xs)}
        row["predicted_config"] = ck.CONFIG_NAMES[ck.config_id(cfg)]
        row["mixed_speedup"] = round(row["mixed"]["solves_per_s"] / row["fp64"]["solves_per_s"], 3)
        rows[name] = row
        Mx.close()
        del b
        log(f"[solvers] {name} done")
    out["cg_async_and_mixed"] = rows

    # -- GMRES(30), convection-diffusion 1024^2 ----------------------------------
    A, xs = W.convdiff_1024()
    Mx = ck.Matrix.from_csr(A, keep_fp32=True)
    b = _rhs(ck, Mx, xs)
    cfg = ck.spmv_select(ck.spmv_features(Mx.handle))
    try:
        ck.spmv_convert(Mx.handle, cfg)
    except ck.CkError as e:
        if e.status != ck.CK_E_UNSUPPORTED:
            raise
        cfg = ck.default_config(Mx.handle)
    row = {"predicted_config": ck.CONFIG_NAMES[ck.config_id(cfg)]}
    xres = {}
    for prec, key in ((ck.CK_PREC_FP64, "fp64"), (ck.CK_PREC_MIXED, "mixed")):
        lat, r, x = _timed_solves(ck, ck.gmres_solve, Mx, b, 1, 1, tol=1e-10, restart=30,
                                  max_iter=200000, precision=prec, config=cfg)
        rr = oracle.relres(A, b.cpu().numpy(), x.cpu().numpy(), parallel=True)
        assert rr <= 1e-10, (key, rr)
        xres[key] = x.cpu().numpy()
        row[key] = {**_lat(lat), "iterations": r["iterations"], "outer_steps": r["outer_steps"],
                    "oracle_true_relres": rr, "forward_error": fe(x, xs)}
    row["mixed_speedup"] = round(row["mixed"]["solves_per_s"] / row["fp64"]["solves_per_s"], 3)
    row["mixed_vs_fp64_rel_diff"] = float(np.linalg.norm(xres["mixed"] - xres["fp64"]) /
                                          np.linalg.norm(xres["fp64"]))
    out["gmres_convdiff_1024"] = row
    Mx.close()
    del b
    log("[solvers] gmres_convdiff_1024 done")

    # -- request loop, shortened trace at tol 1e-10 ------------------------------
    pool = W.serving_pool()
    nreq = args.serve_requests
    Wl = ServingWorkload(pool, nreq, tol=1e-10)
    cap = latency_summary(Wl.run())
    done = Wl.run(arrivals_s=poisson_arrivals(nreq, 0.8 * cap["solves_per_s"], seed=5001))
    st = Wl.stats()
    worst = 0.0
    for c in done:
        t = c["tag"]
        Ap = pool[Wl.mid[t]][0]
        worst = max(worst, oracle.relres(Ap, Wl.b[t].cpu().numpy(), Wl.x[t].cpu().numpy(),
                                         parallel=True))
    out["serve"] = {"requests": nreq, "tol": 1e-10,
                    "closed_loop_solves_per_s": round(cap["solves_per_s"], 3),
                    "arrival_rate_per_s": round(0.8 * cap["solves_per_s"], 3),
                    "solves_per_s": round(st["solves_per_s"], 3),
                    "p50_ms": round(st["p50_latency_us"] * 1e-3, 3),
                    "p99_ms": round(st["p99_latency_us"] * 1e-3, 3),
                    "ok": int(sum(c["status"] == ck.CK_OK for c in done)),
                    "worst_oracle_true_relres": worst,
                    "batched_fraction": round(sum(c["path"] == 0 for c in done) / len(done), 3),
                    "workload": "64-matrix pool (n log-uniform 1e3-1e6), Poisson arrivals at "
                                "0.8x closed-loop capacity, mixed FP32/FP64, CG if symmetric "
                                "else GMRES(30); latency and rate from ck_server_get_stats"}
    Wl.close()
    log("[solvers] serve done")
    return out


# ---------------------------------------------------------------------------
def main():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="spmv_set",
                   choices=["spmv_set", "cg_lap2d", "cg_async", "gmres_mixed", "serve",
                            "select_latency"])
    p.add_argument("--reps", type=int, default=200)
    p.add_argument("--max-n", type=int, default=None, help="drop set members above this n")
    p.add_argument("--only", default=None,
                   help="spmv_set: keep one member, named by its prefix (e.g. uniform_k11); "
                        "for profiling a single matrix, not a bench line")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--table", default=None, help="write the per-matrix timing table (JSON)")
    p.add_argument("--no-table", action="store_true",
                   help="spmv_set: skip the untimed exhaustive and cold tables (profiler runs)")
    p.add_argument("--allocator", default="torch", choices=["torch", "library"],
                   help="spmv_set: where the timed steps' handles take device memory from")
    p.add_argument("--no-solvers", action="store_true",
                   help="spmv_set: skip the untimed solver and serving summary (profiler runs)")
    p.add_argument("--serve-requests", type=int, default=300,
                   help="spmv_set: requests in the solver summary's serving trace")
    p.add_argument("--grid", type=int, default=1024, help="gmres_mixed grid side")
    p.add_argument("--requests", type=int, default=2000, help="serve: requests per trace")
    p.add_argument("--tol", type=float, default=1e-8, help="serve: tolerance")
    p.add_argument("--small-n", type=int, default=8192,
                   help="serve: systems with n <= this run in batched slots")
    p.add_argument("--large-workers", type=int, default=8, help="serve: concurrent large solves")
    p.add_argument("--chunk-iters", type=int, default=8,
                   help="serve: iterations per batched slot per launch")
    p.add_argument("--rate", type=float, default=None,
                   help="serve: fixed arrival rate (solves/s) instead of 0.8x closed-loop capacity")
    args = p.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X (its serving "
              "and solver paths would shard by request, not across GPUs); use --gpus 1.",
              file=sys.stderr)
        return 2
    {"spmv_set": bench_spmv_set, "cg_lap2d": bench_cg_lap2d, "cg_async": bench_cg_async,
     "gmres_mixed": bench_gmres_mixed, "serve": bench_serve,
     "select_latency": bench_select_latency}[args.workload](args)
    return 0


if __name__ == "__main__":
    sys.exit(main())
