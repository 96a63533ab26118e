#!/usr/bin/env python3
"""Benchmark: collision pair-terms/s of the spectral-Galerkin Boltzmann–Nordheim
operator on one MI355X.

Workload (default): 3-D fermions (eps = -1), N = 32^3 Fourier modes, FP64,
hard spheres (Btilde = 4), hbar = 1, L = 8; f0 = 0.45 x a sum of three
Gaussians with seeded centres in |v| <= 2 and variances in [0.3, 1], capped
at 0.99 (seed 0).  One step = one classical RK4 step (four evaluations of
the full operator: forward DFT, classical + W pair sums, outer sum,
trilinear sum, combination, inverse DFT, stage updates) plus the FP64
moments and entropy of the new state.  Kernel-mode tables are built once
when the plan is created, outside the timed region.

value = collision terms per step / seconds per step, where the terms of one
evaluation are the plain Galerkin counts: classical pairs + W pairs + outer
pairs + trilinear triples.

Prints ONE JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

STATS = {-1: "fermions", 0: "classical", 1: "bosons"}
METRIC = "collision pair-terms/s at N=32^3 (FP32c vs FP64); p50/p99 solve latency"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "trilinear_3d32_fp64_hbm_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2110_13735_amd", "csrc", "t1_pairs.hip")
PAIRS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pairs_3d32_hbm_traffic.json")
# the pair-sum kernels and the header that fixes their l-chunking (pair_split)
PAIRS_SOURCE = (os.path.join(ROOT, "paper_2110_13735_amd", "csrc", "collide.hip"),
                os.path.join(ROOT, "paper_2110_13735_amd", "csrc", "bnq_internal.h"))
PEAK_FP64_VALU = 78.6e12  # MI355X dense FP64 vector, FLOP/s
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E, GB/s
PEAK_FP32_VALU = 157.3e12  # MI355X dense FP32 vector, FLOP/s (published; counts packed FP32)
FLOPS_PER_T1_TERM = 4.0   # one real x complex multiply-add (two FMAs)


def cpu_baseline(sample_N: int = 10, nthreads=None):
    """The oracle, untouched, timed on the host: one full evaluation of Qhat
    (direct Galerkin sums, including its own kernel-mode quadrature) of the
    same workload recipe at 3-D N = sample_N."""
    import numpy as np
    import bnq_inputs as inp
    import oracle

    if nthreads:
        os.environ["OMP_NUM_THREADS"] = str(nthreads)
    f = inp.fermion_mixture_3d(N=sample_N, L=8.0, seed=0)
    t0 = time.perf_counter()
    o = oracle.Oracle(3, sample_N)
    o.collide(f, eps=-1, L=8.0)
    dt = time.perf_counter() - t0
    n = sample_N
    h = n // 2
    rng = range(-h, h)
    c1 = sum(1 for l in rng for m in rng if -h <= l + m < h)
    o1 = sum(1 for a in rng for k in rng if -n <= a - k <= n - 2)
    t1 = sum(1 for k in rng for l in rng for m in rng if -h <= k + l + m < h)
    terms = c1 ** 3 + n ** 6 + o1 ** 3 + t1 ** 3
    return {"value": terms / dt, "unit": "pair-terms/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one full oracle evaluation (kernel-mode quadrature + direct sums) of the same recipe "
                      f"at 3-D N={sample_N}: {terms:.3e} terms in {dt:.2f} s"}


def code_hash(*paths):
    """SHA-256 of C/HIP sources (concatenated) with comments and blank space
    removed, so that only a change of the code itself counts."""
    import hashlib
    import re
    src = ""
    for path in paths:
        with open(path) as fh:
            src += fh.read() + "\n"
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = " ".join(src.split())
    return hashlib.sha256(src.encode()).hexdigest()


def measured_traffic():
    """HBM bytes per trilinear launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE counters, or None when the kernel code has changed since the
    counters were taken (the file records the code hash at measurement time)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    if rec.get("kernel_code_sha256") != code_hash(KERNEL_SOURCE):
        return None
    return rec


def measured_pairs_traffic(kernel):
    """The same for a pair-sum kernel (3-D N=32, FP64 or FP32c), keyed by kernel name."""
    if not os.path.exists(PAIRS_TRAFFIC_FILE):
        return None
    with open(PAIRS_TRAFFIC_FILE) as fh:
        rec = json.load(fh).get(kernel)
    if rec is None or rec.get("kernel_code_sha256") != code_hash(*PAIRS_SOURCE):
        return None
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=32)
    ap.add_argument("--dt", type=float, default=None,
                    help="time step (default 0.001 for the 3-D workloads c2, c3 and relax, whose data leave RK4's "
                         "stability region at dt = 0.01; 0.01 for c1, batch and serve)")
    ap.add_argument("--precision", choices=("fp64", "fp32c"), default=None,
                    help="arithmetic of the pair sums (default fp32c for c5, fp64 otherwise)")
    ap.add_argument("--eps", type=int, choices=(-1, 0, 1), default=-1,
                    help="statistics: -1 fermions (default, the trilinear-bound workload), +1 bosons, "
                         "0 classical (only the weight streaming of the pair sums: HBM-bound)")
    ap.add_argument("--schedule", choices=("static", "dynamic"), default="dynamic",
                    help="trilinear work distribution: dynamic (default here, fastest; last bits may vary "
                         "between runs) or static (the library default, bitwise reproducible)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-N", type=int, default=10)
    ap.add_argument("--workload", choices=("c1", "c2", "c3", "relax", "batch", "serve", "c5"), default="c2",
                    help="c2: the 3-D N=32 fermion RK4 step (default); c1: the 2-D N=32 boson RK4 step; "
                         "c3: 3-D bosons near condensation in "
                         "FP32c (--N 32 or 48) with the error against FP64 every 10 steps; relax: the c2 "
                         "trajectory with entropy and distance to its Fermi-Dirac limit every 10 steps; batch: mixed "
                         "instances stepped together; serve: Poisson arrivals (small cells); c5: the serving "
                         "shape N in {16, 24, 32, 48} at 200 req/s in a bounded window, with the sustainable "
                         "rate and a rate sweep on a reduced mix")
    ap.add_argument("--separated", action="store_true",
                    help="c1 only: the trilinear term by the separated-kernel transform route (rank-P kernel "
                         "modes on the doubled grid) instead of the direct sum")
    ap.add_argument("--angles", type=int, default=101,
                    help="c1 --separated: angle count P (101 is the library's default at N=32)")
    ap.add_argument("--instances", type=int, default=60, help="batch workload: number of instances")
    ap.add_argument("--cells", choices=("mixed", "small", "c4"), default="mixed",
                    help="batch workload: cell set (c4: all 18 cells d in {2, 3}, N in {16, 24, 32}, eps in {-1, 0, 1})")
    ap.add_argument("--tuning", default=None,
                    help="batch workload: JSON file of tuned trilinear work distributions (read; with --autotune, "
                         "written)")
    ap.add_argument("--autotune", action="store_true",
                    help="batch workload: autotune the first quantum instance of each cell before batching")
    ap.add_argument("--rate", type=float, default=None,
                    help="serve / c5 workloads: mean arrivals per second (default 10 for serve, 200 for c5)")
    ap.add_argument("--window", type=float, default=150.0, help="c5: wall-clock window of the full-mix run (s)")
    ap.add_argument("--max-service", type=float, default=60.0,
                    help="c5: refuse requests whose estimated service time exceeds this (s)")
    ap.add_argument("--max-active", type=int, default=32, help="c5: most requests served at once")
    ap.add_argument("--sweep", default="0.25,0.5,0.75,1,1.5",
                    help="c5: offered rates (req/s) of the reduced-mix sweep; empty to skip")
    ap.add_argument("--no-sub", action="store_true",
                    help="c2: skip the short FP32c, classical (eps = 0) and serving sub-runs")
    ap.add_argument("--metrics", default=None,
                    help="append JSON lines to this file: every timed step's moments (c2), every request and a "
                         "summary (serve, c5)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run one 1 GiB device copy (read 1 GiB, write 1 GiB) so that a "
                         "counter run can calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one GPU only; multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import bnq_inputs as inp
    import paper_2110_13735_amd as bnq

    if not os.path.exists(bnq.LIBPATH):
        import __graft_entry__
        __graft_entry__.build()
    if args.dt is None:
        args.dt = 0.001 if args.workload in ("c2", "c3", "relax") else 0.01
    if args.rate is None:
        args.rate = 200.0 if args.workload == "c5" else 10.0
    if args.precision is None:
        args.precision = "fp32c" if args.workload == "c5" else "fp64"
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "c5":
        return run_c5(args)
    if args.workload == "c3":
        return run_c3(args)
    if args.workload == "relax":
        return run_relax(args)
    if args.workload == "c1":
        return run_c1(args)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    N, L, eps = args.N, 8.0, args.eps
    prec = bnq.FP32C if args.precision == "fp32c" else bnq.FP64
    sched = bnq.SCHED_DYNAMIC if args.schedule == "dynamic" else bnq.SCHED_STATIC
    p = bnq.Params(d=3, N=N, eps=eps, L=L, precision=prec, schedule=sched)
    f0 = inp.fermion_mixture_3d(N=N, L=L, seed=0)
    t_plan = time.perf_counter()
    plan = bnq.Plan(p)
    t_plan = time.perf_counter() - t_plan
    counts = plan.counts()
    terms_eval = bnq.terms_per_eval(p, counts)
    terms_step = 4.0 * terms_eval
    f = torch.tensor(f0, device=dev)
    stream = torch.cuda.current_stream()

    def one_step():
        # raises (and the bench exits non-zero) when a step's health flags or
        # the moments report a non-finite state or a fermion value >= 1
        plan.step(f, args.dt, bnq.RK4)
        return plan.moments(f, check=True)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mom = None
    log = None
    if args.metrics:
        from paper_2110_13735_amd.metrics import MetricsLog
        log = MetricsLog(args.metrics)
    for k in range(args.steps):
        mom = one_step()
        if log is not None:  # moments() has synchronised: the step is complete
            log.write("step", step=args.warmup + k + 1, t=(args.warmup + k + 1) * args.dt,
                      wall_since_start_s=time.perf_counter() - t0, **mom)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = plan.timing()
    plan.set_timing(False)
    ms_step = 1e3 * elapsed / args.steps
    value = terms_step / (elapsed / args.steps)

    if eps != 0:
        # per evaluation: one launch at N <= 32; larger sums are cut into
        # several launches that together cover the evaluation's terms once
        t1_ms, t1_n = kt["trilinear"]
        evals = 4 * args.steps
        t1_avg_s = (t1_ms / evals) * 1e-3 if t1_n else float("nan")
        flops_launch = counts["trilinear"] * FLOPS_PER_T1_TERM
        achieved = flops_launch / t1_avg_s / 1e12
        tr = measured_traffic() if (prec == bnq.FP64 and eps == -1) else None
        peak = PEAK_FP32_VALU if prec == bnq.FP32C else PEAK_FP64_VALU
        # avg_ms is the trilinear time of one evaluation: one launch at N <= 32
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak / 1e12,
                    "unit": "TFLOP/s", "frac": round(achieved * 1e12 / peak, 4),
                    "traffic": (tr["fetch_bytes"] + tr["write_bytes"]) if tr else None,
                    "kernel": "trilinear_kernel", "avg_ms": round(t1_avg_s * 1e3, 3), "launches": t1_n,
                    "launches_per_eval": t1_n // max(1, evals), "flops_per_eval": flops_launch}
        if tr:
            roofline["traffic_detail"] = {k: tr[k] for k in ("fetch_bytes", "write_bytes", "fetch_scale",
                                                             "write_scale")}
        roofline["measured_peaks"] = measured_peaks(torch, dev)
        roofline["frac_of_measured_fp64_gemm"] = \
            round(achieved / roofline["measured_peaks"]["fp64_gemm_tflops"], 4) if prec == bnq.FP64 else None
    else:
        # classical: the pair sums stream one weight per (l, m) with l + m in I_N
        pr_ms, pr_n = kt["pairs"]
        pr_avg_s = (pr_ms / pr_n) * 1e-3 if pr_n else float("nan")
        bytes_launch = counts["classical"] * (4 if prec == bnq.FP32C else 8)
        achieved = bytes_launch / pr_avg_s / 1e9
        tr = measured_pairs_traffic(f"pairs_kernel<{'float' if prec == bnq.FP32C else 'double'}, false>") \
            if N == 32 else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(achieved / PEAK_HBM_GBS, 4),
                    "traffic": (tr["fetch_bytes"] + tr["write_bytes"]) if tr else None, "kernel": "pairs_kernel",
                    "avg_ms": round(pr_avg_s * 1e3, 4), "launches": pr_n, "bytes_per_launch": bytes_launch}
        roofline["measured_peaks"] = measured_peaks(torch, dev)
        roofline["frac_of_measured_copy"] = round(achieved / roofline["measured_peaks"]["hbm_copy_GB_s"], 4)
    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32c" if prec == bnq.FP32C else "f64",
        "data": "synthetic",
        "config": {"workload": f"3-D {STATS[eps]} eps={eps}, N={N}^3, {args.precision.upper()}, hard spheres, hbar=1, L=8, "
                               f"three-Gaussian f0 (seed 0), RK4 dt={args.dt}, moments every step (dt=0.001: the "
                               f"datum's loss rate ~1e3 puts dt=0.01 outside RK4's stability region; the work per "
                               f"step does not depend on dt)",
                   "d": 3, "N": N, "eps": eps, "precision": args.precision, "schedule": args.schedule,
                   "scheme": "rk4", "dt": args.dt,
                   "terms_per_eval": terms_eval, "evals_per_step": 4,
                   "plan_build_s": round(t_plan, 3)},
        "roofline": roofline,
        "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in kt.items()},
        "moments_last": {k: mom[k] for k in ("rho", "e", "H", "fmax")},
    }
    if eps == -1 and not args.no_sub:
        # short runs of the other figures the metric names, same datum and dt
        out["sub"] = {"fp32c": sub_fp32c(args, plan, f0, terms_eval),
                      "eps0": sub_eps0(args, f0),
                      "latency": sub_latency()}
    plan.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_N)
    print(json.dumps(out))


def sub_fp32c(args, plan64, f0, terms_eval, steps=3):
    """The c2 step in FP32c (FP32 spectra, tables and short sums, FP64 long
    sums, FP64 state) with the mass correction: terms/s, the trilinear
    kernel's fraction of the FP32 peak, the error of Qhat against the FP64
    plan on the initial state, and the mass drift over the steps."""
    import torch
    import paper_2110_13735_amd as bnq

    dev = torch.device("cuda:0")
    p = bnq.Params(d=3, N=args.N, eps=-1, L=8.0, precision=bnq.FP32C, correction=bnq.CORR_MASS,
                   schedule=bnq.SCHED_DYNAMIC if args.schedule == "dynamic" else bnq.SCHED_STATIC)
    plan = bnq.Plan(p)
    f = torch.tensor(f0, device=dev)
    Q = torch.empty_like(f)
    Qh32 = torch.empty(f.shape, dtype=torch.complex128, device=dev)
    Qh64 = torch.empty_like(Qh32)
    plan.collide(f, Q, Qh32)
    plan64.collide(f, Q, Qh64)
    torch.cuda.synchronize()
    qerr = (torch.linalg.norm(Qh32 - Qh64) / torch.linalg.norm(Qh64)).item()
    rho0 = plan.moments(f)["rho"]
    g = f.clone()
    plan.step(g, args.dt, bnq.RK4)  # warm-up on a copy
    torch.cuda.synchronize()
    plan.set_timing(True)
    drift = 0.0
    elapsed = 0.0
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(f, args.dt, bnq.RK4)
        m = plan.moments(f, check=True)
        elapsed += time.perf_counter() - t0
        drift = max(drift, abs(m["rho"] - rho0) / rho0)
    kt = plan.timing()
    plan.set_timing(False)
    plan.close()
    t1_ms, t1_n = kt["trilinear"]
    t1_avg_s = t1_ms / (4 * steps) * 1e-3
    tf = plan64.counts()["trilinear"] * FLOPS_PER_T1_TERM / t1_avg_s / 1e12
    return {"value": 4.0 * terms_eval * steps / elapsed, "unit": "pair-terms/s", "steps": steps,
            "ms_per_step": 1e3 * elapsed / steps, "correction": "mass",
            "trilinear_avg_ms": round(t1_avg_s * 1e3, 3), "trilinear_tflops": round(tf, 3),
            "trilinear_frac_of_fp32_peak": round(tf * 1e12 / PEAK_FP32_VALU, 4),
            "qhat_rel_err_vs_fp64": qerr, "mass_drift_max": drift}


def sub_eps0(args, f0, steps=10):
    """The classical operator (eps = 0) on the same datum, FP64 and FP32c:
    only the pair sums over the classical weight table, an HBM-bound stream;
    roofline of pairs_kernel from its algorithmic bytes (one weight per
    classical pair)."""
    import torch
    import paper_2110_13735_amd as bnq

    dev = torch.device("cuda:0")
    res = {}
    for name, prec in (("fp64", bnq.FP64), ("fp32c", bnq.FP32C)):
        p = bnq.Params(d=3, N=args.N, eps=0, L=8.0, precision=prec)
        plan = bnq.Plan(p)
        terms = bnq.terms_per_eval(p, plan.counts())
        f = torch.tensor(f0, device=dev)
        for _ in range(2):
            plan.step(f, args.dt, bnq.RK4)
        torch.cuda.synchronize()
        plan.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.step(f, args.dt, bnq.RK4)
        plan.moments(f, check=True)
        elapsed = time.perf_counter() - t0
        kt = plan.timing()
        plan.set_timing(False)
        pr_ms, pr_n = kt["pairs"]
        pr_s = pr_ms / pr_n * 1e-3
        nbytes = plan.counts()["classical"] * (4 if prec == bnq.FP32C else 8)
        gbs = nbytes / pr_s / 1e9
        tr = measured_pairs_traffic(f"pairs_kernel<{'float' if prec == bnq.FP32C else 'double'}, false>") \
            if args.N == 32 else None
        res[name] = {"value": 4.0 * terms * steps / elapsed, "unit": "pair-terms/s", "steps": steps,
                     "ms_per_step": 1e3 * elapsed / steps,
                     "roofline": {"bound": "hbm", "kernel": "pairs_kernel", "avg_ms": round(pr_s * 1e3, 4),
                                  "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                  "frac": round(gbs / PEAK_HBM_GBS, 4), "bytes_per_launch": nbytes,
                                  "traffic": (tr["fetch_bytes"] + tr["write_bytes"]) if tr else None}}
        plan.close()
    return res


def sub_latency(n=40, rate=20.0):
    """A short serving run: Poisson arrivals of 3-D requests, N in {8, 12, 16}
    (weights 4:3:2), eps +-1, t_end ~ U[0.05, 0.2] at dt = 0.01: p50/p99
    latency from arrival to completion."""
    from paper_2110_13735_amd import serve
    import bnq_inputs as inp

    reqs = serve.poisson_requests(n, rate=rate, seed=0, cells=[((3, 8), 4), ((3, 12), 3), ((3, 16), 2)],
                                  t_end=(0.05, 0.2))
    srv = serve.Server(lambda r: inp.mixed_instance(r.d, r.N, r.eps, r.seed), budget_bytes=int(64e9), dt=0.01)
    try:
        st = srv.run(reqs)
    finally:
        srv.close()
    return {"requests": n, "rate_per_s": rate, "p50_latency_s": st["p50_latency_s"],
            "p99_latency_s": st["p99_latency_s"], "served_terms_per_s": st["terms_per_s"],
            "completed": st.get("completed"), "failed": st.get("failed")}


def measured_peaks(torch, dev):
    """What this machine sustains right now, beside the published peaks: a 1 GiB
    device copy (read + write bytes / time) and an FP64 GEMM through the vendor
    library (8192^3, 2 flops per multiply-add).  Both run after the timed
    region; they are context for the roofline fraction, not part of the path."""
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    copy_gbs = 2 * a.numel() * 8 * reps / (time.perf_counter() - t0) / 1e9
    del a, b
    n = 8192
    x = torch.rand(n, n, dtype=torch.float64, device=dev)
    y = torch.rand(n, n, dtype=torch.float64, device=dev)
    z = torch.matmul(x, y)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        z = torch.matmul(x, y)
    torch.cuda.synchronize()
    gemm_tf = 2.0 * n ** 3 * reps / (time.perf_counter() - t0) / 1e12
    del x, y, z
    torch.cuda.empty_cache()
    return {"hbm_copy_GB_s": round(copy_gbs, 1), "fp64_gemm_tflops": round(gemm_tf, 2)}


def run_c1(args):
    """2-D bosons (eps = +1), N = 32^2, FP64, Maxwell molecules (B = 1):
    f0 = two isotropic Gaussians at (+-1.5, 0) of variance 0.5, cut at
    |v| <= R = 4 and scaled to mass 1, on [-L, L)^2 with L = (3 + sqrt 2) R / 2;
    one RK4 step of dt per step (four evaluations) plus the moments."""
    import torch

    import bnq_inputs as inp
    import paper_2110_13735_amd as bnq

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    f0, L = inp.two_gaussians_2d(N=32, R_v=4.0)
    sep = args.separated
    p = bnq.Params(d=2, N=32, eps=1, L=L, flags=bnq.FLAG_T1_SEPARATED if sep else 0, angles=args.angles if sep else 0)
    plan = bnq.Plan(p)
    terms_step = 4.0 * bnq.terms_per_eval(p, plan.counts())
    f = torch.tensor(f0, device=dev)
    for _ in range(args.warmup):
        g = f.clone()
        plan.step(g, args.dt, bnq.RK4)
    torch.cuda.synchronize()
    plan.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.step(f, args.dt, bnq.RK4)
        mom = plan.moments(f, check=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = plan.timing()
    plan.set_timing(False)
    t1_ms, t1_n = kt["trilinear"]
    evals = 4 * args.steps
    if sep:
        # per (angle, shift): first-axis transforms of A and B (14 flops per
        # term, M^2 N terms), second axis (16 flops per term, N^2 M terms) and
        # the product (20 flops per output mode)
        Nn, M, P = 32, 64, args.angles
        flops_eval = float(P * M * M * (14 * M * M * Nn + 16 * Nn * Nn * M + 20 * Nn * Nn))
        kernel = "sep_t1_kernel (+ sep_gt, sep_reduce)"
    else:
        flops_eval = plan.counts()["trilinear"] * FLOPS_PER_T1_TERM
        kernel = "trilinear_kernel"
    avg_s = t1_ms / evals * 1e-3
    achieved = flops_eval / avg_s / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                "frac": round(achieved * 1e12 / PEAK_FP64_VALU, 4), "traffic": None, "kernel": kernel,
                "avg_ms": round(avg_s * 1e3, 3), "launches": t1_n, "flops_per_eval": flops_eval}
    out = {
        "metric": METRIC, "value": terms_step * args.steps / elapsed, "unit": "pair-terms/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"2-D bosons eps=+1, N=32^2, FP64, Maxwell molecules, hbar=1, two-Gaussian f0 cut at "
                               f"R=4, L={L:.4f}, RK4 dt={args.dt}"
                               + (f", trilinear term by the separated route with P={args.angles} angles" if sep else ""),
                   "d": 2, "N": 32, "eps": 1, "dt": args.dt, "terms_per_eval": terms_step / 4,
                   "trilinear_route": "separated" if sep else "direct"},
        "roofline": roofline,
        "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in kt.items()},
        "moments_last": {k: mom[k] for k in ("rho", "e", "H", "fmax")},
    }
    plan.close()
    print(json.dumps(out))


def run_relax(args):
    """The c2 trajectory (3-D fermions, N = 32, three-Gaussian f0, RK4) with
    its limit state: the Fermi-Dirac distribution of the same mass, velocity
    and energy (fugacity by Brent's method on eq. eq_fugacity, in the
    library), and every 10 steps the entropy H, the L1 distance and the
    largest pointwise gap to it.  Only the steps are timed."""
    import numpy as np
    import torch

    import bnq_inputs as inp
    import paper_2110_13735_amd as bnq

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    N, L, eps = args.N, 8.0, -1
    prec = bnq.FP32C if args.precision == "fp32c" else bnq.FP64
    sched = bnq.SCHED_DYNAMIC if args.schedule == "dynamic" else bnq.SCHED_STATIC
    p = bnq.Params(d=3, N=N, eps=eps, L=L, precision=prec, schedule=sched)
    plan = bnq.Plan(p)
    terms_step = 4.0 * bnq.terms_per_eval(p, plan.counts())
    f = torch.tensor(inp.fermion_mixture_3d(N=N, L=L, seed=0), device=dev)
    m = plan.moments(f)
    st = bnq.equilibrium(3, eps, 1.0, m["rho"], [m["u0"], m["u1"], m["u2"]], m["e"])
    track = []

    def record(k):
        mk = plan.moments(f, check=False)
        dk = plan.equilibrium_distance(f, st)
        track.append({"step": k, "t": round(k * args.dt, 6), "H": mk["H"], "l1": dk["l1"], "max_abs": dk["max_abs"],
                      "fmax": mk["fmax"], "rho": mk["rho"], "e": mk["e"]})
        print(f"relax step {k}: H {mk['H']:.8f} L1 {dk['l1']:.4e}", file=sys.stderr, flush=True)

    record(0)
    elapsed = 0.0
    for k in range(1, args.steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(f, args.dt, bnq.RK4)
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        if k % 10 == 0 or k == args.steps:
            record(k)
    out = {
        "metric": METRIC,
        "value": terms_step * args.steps / elapsed,
        "unit": "pair-terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 0,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32c" if prec == bnq.FP32C else "f64",
        "data": "synthetic",
        "config": {"workload": f"3-D fermions eps=-1, N={N}^3, {args.precision.upper()}, hard spheres, hbar=1, L=8, "
                               f"three-Gaussian f0 (seed 0), RK4 dt={args.dt} to t={args.steps * args.dt:g}, "
                               f"relaxation to the Fermi-Dirac limit tracked every 10 steps",
                   "d": 3, "N": N, "eps": eps, "precision": args.precision, "dt": args.dt},
        "limit_state": st.as_dict(),
        "relaxation": track,
    }
    plan.close()
    print(json.dumps(out))


def run_c3(args):
    """3-D bosons (eps = +1) near condensation, f0 = a exp(-|v|^2 / T) with
    T = 0.2, a = 10.6, L = 3: RK4 steps with the pair sums and the trilinear
    sum in FP32c (FP32 spectra and tables, FP32 sums of at most two inner
    rows, FP64 totals), the tables computed in FP64 and rounded, the moments
    and stage updates in FP64.  Only the FP32c steps are timed.  At N = 32 an
    FP64 trajectory runs beside it (untimed), and every 10 steps the bench
    records the relative error of the FP32c Qhat on the current state and of
    the moments of the FP32c trajectory against it; at N = 48 the FP64 tables
    (364 GB) do not fit one GPU and only the FP32c run is made.  The datum's
    limit state is a condensate (ratio beyond the end of I_eq); every 10 steps
    the run also records the L1 distance to its z = 1 part and the mass at the
    node v = u, where the condensed mass m0 gathers."""
    import numpy as np
    import torch

    import bnq_inputs as inp
    import paper_2110_13735_amd as bnq

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    N, L, eps = args.N, 3.0, 1
    sched = bnq.SCHED_DYNAMIC if args.schedule == "dynamic" else bnq.SCHED_STATIC
    p32 = bnq.Params(d=3, N=N, eps=eps, L=L, precision=bnq.FP32C, schedule=sched, correction=bnq.CORR_MASS)
    f0 = inp.boson_condensing_3d(N=N, L=L)
    t_plan = time.perf_counter()
    plan = bnq.Plan(p32)
    t_plan = time.perf_counter() - t_plan
    terms_step = 4.0 * bnq.terms_per_eval(p32, plan.counts())
    ref = None
    if N <= 32:
        ref = bnq.Plan(bnq.Params(d=3, N=N, eps=eps, L=L, schedule=sched))
    f = torch.tensor(f0, device=dev)
    g = torch.tensor(f0, device=dev)
    Q32 = torch.empty_like(f)
    Q64 = torch.empty_like(f)
    Qh32 = torch.empty(f.shape, dtype=torch.complex128, device=dev)
    Qh64 = torch.empty_like(Qh32)
    checks = []
    # the limit state of the datum's moments: a condensate (z = 1 plus the
    # mass m0 at v = u) for this supercritical ratio
    m0 = plan.moments(f, check=False)
    lim = bnq.equilibrium(3, eps, 1.0, m0["rho"], [m0["u0"], m0["u1"], m0["u2"]], m0["e"])
    relax = []

    def track(step):
        dk = plan.equilibrium_distance(f, lim)
        relax.append({"step": step, "l1_regular_part": dk["l1"], "mass_at_v_eq_u": dk["mass_excluded"],
                      "fmax": plan.moments(f, check=False)["fmax"]})

    def check(step):
        if ref is None:
            return
        plan.collide(f, Q32, Qh32)
        ref.collide(f, Q64, Qh64)
        m32, m64 = plan.moments(f, check=False), ref.moments(g, check=False)
        torch.cuda.synchronize()
        eq = (torch.linalg.norm(Qh32 - Qh64) / torch.linalg.norm(Qh64)).item()
        em = {k: abs(m32[k] - m64[k]) / max(abs(m64[k]), 1e-300) for k in ("rho", "e", "H", "fmax")}
        checks.append({"step": step, "qhat_rel_err": eq, "moments_rel_err": em})
        print(f"c3 N={N} step {step}: FP32c Qhat error {eq:.2e}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):  # warm-up steps act on copies of the start state
        h = f.clone()
        plan.step(h, args.dt, bnq.RK4)
    torch.cuda.synchronize()
    check(0)
    track(0)
    elapsed = 0.0
    blow_up = None
    for k in range(1, args.steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(f, args.dt, bnq.RK4)
        m = plan.moments(f, check=False)
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        if m["status"] == bnq.BNQ_ENONFINITE:
            blow_up = k
            break
        print(f"c3 N={N} step {k}: {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
        if ref is not None:
            ref.step(g, args.dt, bnq.RK4)
        if k % 10 == 0 or k == args.steps:
            check(k)
            track(k)
    if blow_up:
        print(f"c3: non-finite state after step {blow_up}", file=sys.stderr, flush=True)
    mom = plan.moments(f, check=False)
    out = {
        "metric": METRIC,
        "value": terms_step * (blow_up or args.steps) / elapsed,
        "unit": "pair-terms/s",
        "n_gpus": 1,
        "steps": blow_up or args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / (blow_up or args.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32c",
        "data": "synthetic",
        "config": {"workload": f"3-D bosons eps=+1 near condensation, N={N}^3, FP32c pair and trilinear sums, "
                               f"FP64 tables precompute, moments and RK4 stages (dt={args.dt}); "
                               f"f0 = 10.6 exp(-|v|^2/0.2), L=3, hard spheres",
                   "d": 3, "N": N, "eps": eps, "precision": "fp32c", "schedule": args.schedule,
                   "terms_per_eval": terms_step / 4, "plan_build_s": round(t_plan, 3)},
        "error_vs_fp64": checks if ref is not None else
        "FP64 tables (364 GB) do not fit one GPU at N=48; FP32c parity is checked on sparse spectra",
        "moments_last": {k: mom[k] for k in ("rho", "e", "H", "fmax")},
        "limit_state": lim.as_dict(),
        "relaxation": relax,
        "blow_up_step": blow_up,
    }
    plan.close()
    if ref is not None:
        ref.close()
    print(json.dumps(out))


BATCH_CELLS = {"mixed": [(2, 16), (2, 24), (2, 32), (3, 16), (3, 24)],
               "small": [(2, 8), (2, 16), (2, 24), (3, 8), (3, 12)],
               "c4": [(2, 16), (2, 24), (2, 32), (3, 16), (3, 24), (3, 32)]}


def run_batch(args):
    """Mixed instances (d, N, eps) advanced together: one batched RK4 step per
    step (HIP graph replay), against the same instances stepped one after the
    other through their own plans.  Both runs start from the same states and
    take the same steps; the final states must agree bitwise."""
    import numpy as np
    import torch

    import bnq_inputs as inp
    import paper_2110_13735_amd as bnq

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cell_set = BATCH_CELLS[args.cells]
    cells = [(d, N, e) for (d, N) in cell_set for e in (-1, 0, 1)]
    prec = bnq.FP32C if args.precision == "fp32c" else bnq.FP64
    sched = bnq.SCHED_DYNAMIC if args.schedule == "dynamic" else bnq.SCHED_STATIC
    if args.tuning and os.path.exists(args.tuning) and not args.autotune:
        _progress(f"tuning records loaded: {bnq.load_tuning(args.tuning)}")
    plans, f_b, f_s, terms = [], [], [], 0.0
    tuned, tune_ms, tuned_pairs = set(), {}, {}
    for i in range(args.instances):
        if i and i % 64 == 0:
            _progress(f"{i} plans created")
        d, N, eps = cells[i % len(cells)]
        f0, L = inp.mixed_instance(d, N, eps, seed=i)
        p = bnq.Params(d=d, N=N, eps=eps, L=L, precision=prec, schedule=sched,
                       correction=bnq.CORR_MASS if prec == bnq.FP32C else bnq.CORR_NONE)
        pl = bnq.Plan(p)
        if args.autotune and eps != 0 and (d, N, prec) not in tuned:
            # the first quantum instance of a cell picks the work distribution;
            # plans created afterwards start with the recorded choice
            ch, ms = pl.autotune(torch.tensor(f0, device=dev), reps=2)
            tuned.add((d, N, prec))
            tune_ms[(d, N, prec)] = ms
            _progress(f"autotune ({d}, {N}): choice {ch}, ms {np.round(ms, 3).tolist()}")
        if args.autotune and (d, N, prec, int(eps == 0)) not in tuned_pairs:
            # likewise the pair-sum l-chunking, once per cell and eps == 0 or not
            sp, ms = pl.autotune_pairs(torch.tensor(f0, device=dev), reps=3)
            tuned_pairs[(d, N, prec, int(eps == 0))] = (eps, ms)
            _progress(f"pair autotune ({d}, {N}, eps={eps}): split {sp}, ms {np.round(ms, 3).tolist()}")
        plans.append(pl)
        terms += 4.0 * bnq.terms_per_eval(p, pl.counts())
        f_b.append(torch.tensor(f0, device=dev))
        f_s.append(torch.tensor(f0, device=dev))
    if args.autotune and args.tuning:
        pc = {(d, N, pr, e): ms for (d, N, pr, _), (e, ms) in tuned_pairs.items()}
        _progress(f"tuning records saved: "
                  f"{bnq.save_tuning(args.tuning, sorted(tuned), tune_ms, pair_cells=sorted(pc), pair_ms=pc)}")
    dt = args.dt
    stream = torch.cuda.Stream()
    batch = bnq.Batch(plans, f_b)
    layout = batch.layout()
    torch.cuda.synchronize()
    _progress(f"{len(plans)} plans, {len(cells)} cells, {terms:.3e} terms per step; "
              f"{layout[0]} groups, {layout[1]} shared trilinear launch(es) per stage")

    def solo_step():
        for j, (pl, f) in enumerate(zip(plans, f_s)):
            pl.step(f, dt)
            if len(plans) > 144 and (j + 1) % 64 == 0:
                torch.cuda.synchronize()
                _progress(f"solo: {j + 1} of {len(plans)} instances stepped")

    for w in range(args.warmup):
        batch.step(dt, bnq.RK4, graph=True, stream=stream)
        stream.synchronize()  # the plans' workspaces serve both runs: never overlap them
        solo_step()
        torch.cuda.synchronize()
        _progress(f"warmup step {w + 1} done")
    t0 = time.perf_counter()
    for k in range(args.steps):
        batch.step(dt, bnq.RK4, graph=True, stream=stream)
        if args.steps > 1:
            stream.synchronize()
            _progress(f"batched step {k + 1}: {time.perf_counter() - t0:.1f} s")
    stream.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    _progress(f"batched: {t_batch:.3f} s per step")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        solo_step()
        if args.steps > 1:
            torch.cuda.synchronize()
            _progress(f"solo step {k + 1}: {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    t_solo = (time.perf_counter() - t0) / args.steps
    same = all(torch.equal(a, b) for a, b in zip(f_b, f_s))
    rel = max((torch.linalg.norm(a - b) / torch.linalg.norm(b)).item() for a, b in zip(f_b, f_s))
    batch.close()
    for pl in plans:
        pl.close()
    out = {
        "metric": "collision pair-terms/s, mixed instances stepped together (aggregate)",
        "value": terms / t_batch,
        "unit": "pair-terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_batch,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32c" if args.precision == "fp32c" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.instances} instances over cells (d, N) in {cell_set} x eps in (-1, 0, 1), "
                               f"Gaussian-mixture data (seed = instance), RK4 dt={dt}, one HIP-graph replay per step",
                   "instances": args.instances, "terms_per_step": terms, "schedule": args.schedule,
                   "groups": layout[0], "shared_trilinear_launches_per_stage": layout[1],
                   "tuning": {f"{d}d{N}": bnq.tune_get(d, N, prec) for (d, N) in cell_set},
                   "pair_split": {f"{d}d{N}" + ("eps0" if e == 0 else ""): bnq.tune_pairs_get(d, N, prec, e)
                                  for (d, N, e) in cells}},
        "solo": {"value": terms / t_solo, "ms_per_step": 1e3 * t_solo, "speedup": t_solo / t_batch},
        "bitwise_equal_to_solo": bool(same),
        "max_rel_diff_vs_solo": rel,
    }
    print(json.dumps(out))


def run_serve(args):
    """Poisson arrivals served by continuous batching: 3-D requests with
    N in {8, 12, 16} (weights 4:3:2), eps in {-1, +1}, t_end ~ U[0.05, 0.5]
    (RK4, dt = 0.01), Gaussian-mixture data; p50/p99 latency from arrival to
    completion and the terms/s actually served."""
    from paper_2110_13735_amd import serve
    import bnq_inputs as inp

    reqs = serve.poisson_requests(args.instances, rate=args.rate, seed=0,
                                  cells=[((3, 8), 4), ((3, 12), 3), ((3, 16), 2)], t_end=(0.05, 0.5))
    import paper_2110_13735_amd as bnq

    prec = bnq.FP32C if args.precision == "fp32c" else bnq.FP64
    srv = serve.Server(lambda r: inp.mixed_instance(r.d, r.N, r.eps, r.seed), budget_bytes=int(64e9), dt=args.dt,
                       precision=prec)
    log = None
    if args.metrics:
        from paper_2110_13735_amd.metrics import MetricsLog
        log = MetricsLog(args.metrics)
    try:
        st = srv.run(reqs, metrics=log)
    finally:
        srv.close()
    out = {
        "metric": "served collision pair-terms/s; p50/p99 solve latency",
        "value": st["terms_per_s"], "unit": "pair-terms/s", "n_gpus": 1, "steps": st["ticks"], "warmup": 0,
        "ms_per_step": 1e3 * st["busy_s"] / max(1, st["ticks"]), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32c" if prec == bnq.FP32C else "f64", "data": "synthetic",
        "config": {"workload": f"{args.instances} Poisson arrivals at {args.rate} req/s, 3-D N in (8, 12, 16) "
                               f"weights 4:3:2, eps +-1, t_end U[0.05, 0.5], RK4 dt={args.dt}",
                   "rate_per_s": args.rate},
        "p50_latency_s": st["p50_latency_s"], "p99_latency_s": st["p99_latency_s"],
        "serve": st,
    }
    print(json.dumps(out))


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_c5(args):
    """The serving shape: Poisson arrivals at 200 req/s of 3-D solves, N in
    {16, 24, 32, 48} (weights 4:3:2:1), eps in {-1, +1}, t_end ~ U[0.5, 5] at
    dt = 0.01, mixed Gaussian data, FP32c.

    1. Calibration: device seconds per RK4 step of one lone request at
       N = 16, 24, 32 (measured); N = 48 from N = 32 by the growth of the
       trilinear term count, (48/32)^9.
    2. The first 256 arrivals served for a bounded wall-clock window, with
       requests whose estimated service time exceeds --max-service refused:
       offered against achieved load (device seconds per second), completions
       and p50/p99 latency of what completed, and the rate the full mix could
       sustain (1 / mean service time).
    3. A rate sweep on a reduced mix (N in {16, 24}, weights 4:1, t_end ~
       U[0.05, 0.2]): latency and achieved load per offered rate, arrivals
       over about 40 s each, at most 60 s per rate."""
    import collections

    import numpy as np
    import torch

    from paper_2110_13735_amd import serve
    import bnq_inputs as inp
    import paper_2110_13735_amd as bnq

    prec = bnq.FP32C if args.precision == "fp32c" else bnq.FP64
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    make = lambda r: inp.mixed_instance(r.d, r.N, r.eps, r.seed)  # noqa: E731
    cost = {}
    for N in (16, 24, 32):
        f0, L = inp.mixed_instance(3, N, -1, 99)
        with bnq.Plan(bnq.Params(d=3, N=N, eps=-1, L=L, precision=prec)) as pl:
            f = torch.tensor(f0, device=dev)
            pl.step(f, args.dt)
            torch.cuda.synchronize()
            k = 4 if N < 32 else 1
            t0 = time.perf_counter()
            for _ in range(k):
                pl.step(f, args.dt)
            torch.cuda.synchronize()
            cost[N] = (time.perf_counter() - t0) / k
        _progress(f"calibration: 3-D N={N}: {cost[N]:.4g} s per RK4 step")
    cost[48] = cost[32] * 1.5 ** 9
    step_cost = lambda r: cost[r.N]  # noqa: E731
    log = None
    if args.metrics:
        from paper_2110_13735_amd.metrics import MetricsLog
        log = MetricsLog(args.metrics)
        log.write("calibration", s_per_step={f"3d{k}": v for k, v in cost.items()})

    def nsteps(r):
        return max(1, int(math.ceil(r.t_end / args.dt - 1e-9)))

    def hook_every(reqs, period):
        last = [0.0]

        def hook(srv, now):
            if now - last[0] >= period:
                last[0] = now
                _progress(f"t={now:.0f}s done={sum(r.status == 'done' for r in reqs)} "
                          f"active={sum(r.status == 'active' for r in reqs)}")
        return hook

    def serve_run(reqs, max_wall, max_service):
        srv = serve.Server(make, budget_bytes=int(200e9), dt=args.dt, precision=prec, max_service_s=max_service,
                           step_cost=step_cost, max_active=args.max_active)
        try:
            st = srv.run(reqs, max_wall=max_wall, on_tick=hook_every(reqs, 15.0), metrics=log)
        finally:
            srv.close()
        span = max(r.arrival for r in reqs)
        offered = sum(nsteps(r) * cost[r.N] for r in reqs) / max(span, 1e-9)
        st["offered_device_s_per_s"] = offered
        st["achieved_device_s_per_s"] = st["busy_s"] / st["elapsed_s"]
        st["arrival_span_s"] = span
        return st

    # 2. the full mix
    cells = [((3, 16), 4), ((3, 24), 3), ((3, 32), 2), ((3, 48), 1)]
    reqs = serve.poisson_requests(256, rate=args.rate, seed=0, cells=cells, t_end=(0.5, 5.0))
    mean_service = sum(nsteps(r) * cost[r.N] for r in reqs) / len(reqs)
    _progress(f"full mix: 256 arrivals at {args.rate} req/s, mean service {mean_service:.1f} s, "
              f"window {args.window} s")
    full = serve_run(reqs, args.window, args.max_service)
    per_cell = {}
    for N in (16, 24, 32, 48):
        rs = [r for r in reqs if r.N == N]
        per_cell[f"3d{N}"] = {"arrivals": len(rs), "completed": sum(r.status == "done" for r in rs),
                              "refused": sum(r.status == "refused" for r in rs),
                              "failed": sum(r.status == "failed" for r in rs),
                              "failed_eps": dict(collections.Counter(r.eps for r in rs if r.status == "failed")),
                              "failed_steps_mean": float(np.mean([r.steps for r in rs if r.status == "failed"]))
                              if any(r.status == "failed" for r in rs) else None,
                              "est_service_s_mean": float(np.mean([nsteps(r) * cost[N] for r in rs])) if rs else 0}
    full["per_cell"] = per_cell
    # 3. the reduced-mix sweep
    reduced = [((3, 16), 4), ((3, 24), 1)]
    sweep = []
    for rate in [float(x) for x in args.sweep.split(",") if x.strip()]:
        n = max(8, int(round(rate * 40)))
        rs = serve.poisson_requests(n, rate=rate, seed=1, cells=reduced, t_end=(0.05, 0.2))
        _progress(f"sweep: {n} arrivals at {rate} req/s")
        st = serve_run(rs, 60.0, None)
        sweep.append({"rate_per_s": rate, "requests": n, "completed": st["completed"],
                      "unfinished": st["unfinished"], "p50_latency_s": st["p50_latency_s"],
                      "p99_latency_s": st["p99_latency_s"], "offered_device_s_per_s": st["offered_device_s_per_s"],
                      "achieved_device_s_per_s": st["achieved_device_s_per_s"], "terms_per_s": st["terms_per_s"]})
    red = serve.poisson_requests(1000, rate=1.0, seed=1, cells=reduced, t_end=(0.05, 0.2))
    out = {
        "metric": "served collision pair-terms/s; p50/p99 solve latency (serving shape)",
        "value": full["terms_per_s"], "unit": "pair-terms/s", "n_gpus": 1, "steps": full["ticks"], "warmup": 0,
        "ms_per_step": 1e3 * full["busy_s"] / max(1, full["ticks"]), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32c" if prec == bnq.FP32C else "f64", "data": "synthetic",
        "config": {"workload": f"first 256 Poisson arrivals at {args.rate} req/s, 3-D N in (16, 24, 32, 48) "
                               f"weights 4:3:2:1, eps +-1, t_end U[0.5, 5], RK4 dt={args.dt}, mixed Gaussian data; "
                               f"{args.window} s window, at most {args.max_active} served at once, refusal above "
                               f"{args.max_service} s estimated service",
                   "rate_per_s": args.rate},
        "p50_latency_s": full["p50_latency_s"], "p99_latency_s": full["p99_latency_s"],
        "calibration_s_per_step": {f"3d{k}": v for k, v in cost.items()},
        "full_mix_mean_service_s": mean_service, "full_mix_sustainable_rate_per_s": 1.0 / mean_service,
        "reduced_mix_sustainable_rate_per_s": 1.0 / (sum(nsteps(r) * cost[r.N] for r in red) / len(red)),
        "serve": full, "sweep": sweep,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
