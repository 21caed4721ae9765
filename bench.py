#!/usr/bin/env python3
"""Benchmark of the FS-1 hot path on one MI355X.

A step is one full solve of the single-pair log-domain workload: N = 2^20 grid
points on [0, 1] (h = 1/N), Gaussian-mixture marginals with 3-5 components,
eps = 1e-3, stop at an L1 marginal error <= 1e-8 or 5000 iterations.  Every step
runs the whole path: validation and set-up, the half-iteration kernels (scans,
fused update, stopping-test error), the final marginal errors and the transport
cost.  Inputs are resident in device memory before the timed region.

Output: one JSON line (stdout).  `value` is grid-points x iterations per second
over the timed steps.  `roofline` describes the dominant kernel (the
half-iteration update), timed with HIP events on the solve stream inside the
timed region.  `cpu_baseline` times the CPU oracle (the sequential FS-1 of
Algorithm 1 in the log domain, one core) on a bounded sample of the same
workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f64|f32]
       python bench.py --copy-calibration   (plain copy of known size, for the
                                             hardware-counter traffic scale)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak, GB/s (vendor figure)
PROFILE_STRIDE = 4             # time every 4th polling batch of update kernels
N_C2 = 1 << 20
SEED = 1
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fused_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2202_10042_amd", "csrc", f)
                  for f in ("fs1_fused.hip", "fs1_frame.h", "fs1_device.h", "fs1_internal.h",
                            "fs1_tile.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(dtype: str, workload: str):
    """Per-launch HBM/fabric traffic of the half-iteration kernel from the
    committed counter summary, or None when the kernel changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    e = t.get("entries", {}).get(f"{workload}:{dtype}")
    return None if e is None else e.get("bytes_per_launch")


def copy_calibration(mib: int = 1024):
    """Plain device-to-device copy of a known size (read mib MiB, write mib MiB)."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    gbs = 2 * n * 8 / dt / 1e9
    log(f"copy {mib} MiB: {dt * 1e3:.3f} ms, {gbs:.1f} GB/s (read+write)")
    return gbs


def cpu_baseline(mu, nu, h, eps, iters: int):
    """The CPU oracle as it stands: sequential log-domain FS-1, one core."""
    import oracle
    t0 = time.perf_counter()
    r = oracle.fs1_log(mu, nu, h, eps, tol=0.0, itr_max=iters)
    dt = time.perf_counter() - t0
    return {"value": mu.size * r.iterations / dt, "unit": "grid-points*iterations/s",
            "cores": 1, "kind": "oracle",
            "sample": f"oracle.fs1_log (sequential log-domain Algorithm 1, binary64) on the "
                      f"same N={mu.size} eps={eps} inputs, {r.iterations} fixed iterations "
                      f"(tol 0), {dt:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--itr-max", type=int, default=5000)
    ap.add_argument("--n", type=int, default=N_C2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=80)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="a 256 MiB device copy, then one fixed 300-iteration solve of the "
                         "workload (for hardware-counter runs)")
    ap.add_argument("--large", action="store_true",
                    help="also run the N=1e8 eps=1e-4 precision-study solve (f64 and f32)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 4096-instance uneven batch (binary32, tol 1e-6)")
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the Poisson request stream through the server")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--no-paper-workloads", action="store_true",
                    help="skip the Sec. 5.1 / 5.2 / 5.3 workloads at the paper's sizes")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); libfs1 has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2202_10042_amd import fs1, inputs
    if not os.path.exists(fs1.LIB_PATH):
        from paper_2202_10042_amd import build
        build.build()

    if args.copy_calibration:
        copy_calibration()
        return

    n = args.n
    k = inputs.random_k(SEED)
    mu_np, nu_np = inputs.mixture_pair(n, k, SEED)
    h = 1.0 / n
    mu = torch.tensor(mu_np, dtype=torch.float64, device="cuda")
    nu = torch.tensor(nu_np, dtype=torch.float64, device="cuda")
    ctx = fs1.Context(torch.cuda.current_stream())
    if args.traffic_probe:
        copy_calibration(256)
        r = fs1.fs1_solve(mu, nu, args.eps, 0.0, itr_max=300, dtype=args.dtype, domain="log",
                          sync_every=64, ctx=ctx)
        torch.cuda.synchronize()
        log(f"probe solve: {r.iterations} iterations, w1 {r.w1:.12g}")
        return

    def solve(dtype, eps, itr_max=args.itr_max, tol=args.tol, m=mu, v=nu):
        return fs1.fs1_solve(m, v, eps, tol, itr_max=itr_max, dtype=dtype, domain="log",
                             sync_every=64, ctx=ctx)

    log(f"workload: N={n} K={k} eps={args.eps} tol={args.tol} itr_max={args.itr_max} "
        f"dtype={args.dtype}")
    for _ in range(args.warmup):
        r = solve(args.dtype, args.eps)
        log(f"warmup: iterations {r.iterations} err {r.marginal_err:.3e} w1 {r.w1:.12g}")

    ctx.set_profiling(PROFILE_STRIDE)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    its = 0
    res = None
    ev0.record()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = solve(args.dtype, args.eps)
        its += res.iterations
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    kms, klaunch, kbytes = ctx.kernel_stats()
    ctx.set_profiling(0)
    if res is None or res.status != 0:
        print(f"solve failed: {res}", file=sys.stderr)
        sys.exit(1)
    ms_per_step = wall * 1e3 / args.steps
    value = n * its / wall
    log(f"timed: {args.steps} solves, {its} iterations, {wall:.3f} s wall ({gpu_ms:.1f} ms "
        f"stream), {ms_per_step:.2f} ms/solve, {value:.4g} grid-pts*it/s, "
        f"{wall / max(its, 1) * 1e6:.2f} us/iteration")
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else None
    avg_us = kms * 1e3 / klaunch if klaunch else None
    log(f"half-iteration kernel: {klaunch} launches, avg {avg_us:.2f} us, "
        f"{achieved:.1f} GB/s algorithmic")
    workload = "c2"
    traffic = measured_traffic(args.dtype, workload)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": "fs1::k_fused (psi and phi halves)",
                "avg_launch_us": round(avg_us, 3), "launches": klaunch,
                "alg_bytes_per_launch": round(kbytes / klaunch)}

    out = {
        "metric": "grid-points*iterations/s",
        "value": value,
        "unit": "grid-points*iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded Gaussian-mixture histograms)",
        "config": {
            "workload": "single pair, log-domain stabilised FS-1, N=2^20 uniform grid on "
                        "[0,1], 3-5 component Gaussian mixtures, eps=1e-3, tol 1e-8, "
                        "itr_max 5000",
            "n": n, "eps": args.eps, "tol": args.tol, "itr_max": args.itr_max,
            "mixture_components": k, "seed": SEED, "domain": "log", "check_every": 1,
            "iterations_per_solve": res.iterations, "converged": res.converged,
            "marginal_err": res.marginal_err, "w1": res.w1,
        },
        "roofline": roofline,
    }

    if not args.no_variants:
        variants = []
        for dt in ("f64", "f32"):
            for eps in (1e-3, 1e-4):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = solve(dt, eps)
                torch.cuda.synchronize()
                w = time.perf_counter() - t0
                variants.append({"dtype": dt, "eps": eps, "iterations": r.iterations,
                                 "converged": r.converged, "marginal_err": r.marginal_err,
                                 "w1": r.w1, "ms": round(w * 1e3, 2),
                                 "grid_pts_it_per_s": n * r.iterations / w})
                log(f"variant {dt} eps={eps}: {r.iterations} it, err {r.marginal_err:.3e}, "
                    f"w1 {r.w1:.12g}, {w * 1e3:.1f} ms")
        # the same workload in the other solvers: the threshold-absorption
        # variant (tau = 1e3, general path) and the single-launch persistent one
        for label, kw in (("absorb tau=1e3", dict(domain="absorb", tau=1e3)),
                          ("persistent", dict(domain="log", solver="persistent"))):
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = fs1.fs1_solve(mu, nu, args.eps, args.tol, itr_max=args.itr_max, dtype="f64",
                                  sync_every=64, ctx=ctx, **kw)
                torch.cuda.synchronize()
                w = time.perf_counter() - t0
            variants.append({"dtype": "f64", "eps": args.eps, "solver": label,
                             "iterations": r.iterations, "converged": r.converged,
                             "marginal_err": r.marginal_err, "w1": r.w1,
                             "absorptions": r.absorptions, "ms": round(w * 1e3, 2),
                             "grid_pts_it_per_s": n * r.iterations / w})
            log(f"variant {label}: {r.iterations} it, err {r.marginal_err:.3e}, "
                f"w1 {r.w1:.12g}, {w * 1e3:.1f} ms")
        out["variants"] = variants

    if args.large:
        out["large_n"] = large_n_study(fs1, ctx, inputs, np, torch)

    if not args.no_batched:
        out["batched"] = batched_study(fs1, ctx, inputs, np, torch, args.batch)

    if not args.no_serving:
        out["serving"] = serving_study(fs1, ctx, inputs, np, torch, args.serve_seconds)

    if not args.no_paper_workloads:
        out["paper_workloads"] = paper_workloads_study(fs1, ctx, inputs, np, torch)

    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle.fs1_log, {args.cpu_iters} iterations at N={n} ...")
        out["cpu_baseline"] = cpu_baseline(mu_np, nu_np, h, args.eps, args.cpu_iters)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.4g} grid-pts*it/s")

    print(json.dumps(out), flush=True)


# The paper's FS-1 and dense Sinkhorn times (seconds per solve, its CPU; Sec. 5,
# Tables 1 and 2), quoted as context for the GPU times on the same workloads.
PAPER_TIMES = {
    "table1": {500: (8.70e-3, 7.68e-2), 2000: (4.25e-2, 2.81e0), 8000: (1.53e-1, 4.80e1)},
    "table2": {500: (4.90e-3, 2.30e-2), 2000: (1.52e-2, 1.36e0), 8000: (5.96e-2, 2.81e1)},
    # Sec. 5.3, Table 3 (N x N grids)
    "table3": {10: (1.27e-2, 8.02e-2), 20: (2.01e-2, 6.73e-1), 40: (7.38e-2, 1.38e1),
               80: (2.64e-1, 4.78e2), 160: (1.08e0, 1.38e4)},
}


def paper_workloads_study(fs1, ctx, inputs, np, torch):
    """Sec. 5.1 (uniform random marginals on [-3, 3], eps = 1e-3, 1000
    iterations) and Sec. 5.2 (Ricker wavelets, eps = 1e-2, 500 iterations) at
    N = 500, 2000, 8000: binary64 solves with a fixed iteration count, plain
    (as in the paper), log domain and the threshold-absorption variant (tau =
    1e3); best of three timed solves each."""
    spec = {"table1": (lambda n: inputs.paper_uniform_pair(n, 0), 1e-3, 1000),
            "table2": (lambda n: inputs.ricker_pair(n), 1e-2, 500)}
    rows = []
    for name, (gen, eps, its) in spec.items():
        for n in (500, 2000, 8000):
            u, v, h = gen(n)
            mu = torch.tensor(u, dtype=torch.float64, device="cuda")
            nu = torch.tensor(v, dtype=torch.float64, device="cuda")
            for domain in ("plain", "log", "absorb"):
                best, r = None, None
                for rep in range(4):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    r = fs1.fs1_solve(mu, nu, eps, 0.0, h=h, itr_max=its, dtype="f64",
                                      domain=domain, sync_every=64, ctx=ctx)
                    torch.cuda.synchronize()
                    w = time.perf_counter() - t0
                    if rep > 0:
                        best = w if best is None else min(best, w)
                pf, pd = PAPER_TIMES[name][n]
                rows.append({"workload": name, "n": n, "eps": eps, "iterations": r.iterations,
                             "domain": domain, "status": r.status, "w1": r.w1,
                             "absorptions": r.absorptions,
                             "marginal_err": r.marginal_err, "gpu_s": best,
                             "paper_fs1_cpu_s": pf, "paper_dense_cpu_s": pd,
                             "speedup_vs_paper_fs1": pf / best})
                log(f"{name} n={n} {domain}: {r.iterations} it, {best * 1e3:.2f} ms per solve "
                    f"(paper's FS-1 on its CPU: {pf * 1e3:.1f} ms), w1 {r.w1:.12g}")
    # Sec. 5.3: uniform random marginals on N x N grids, h1 = h2 = 1, eps = 0.01,
    # 1000 iterations, Algorithm 2 (plain binary64)
    for n in (10, 20, 40, 80, 160):
        u, v = inputs.paper_uniform_2d(n, n, 0)
        mu = torch.tensor(u, dtype=torch.float64, device="cuda")
        nu = torch.tensor(v, dtype=torch.float64, device="cuda")
        best, r = None, None
        for rep in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fs1.fs1_solve_2d(mu, nu, n, n, 1.0, 1.0, 0.01, 0.0, itr_max=1000, sync_every=64,
                                 ctx=ctx)
            torch.cuda.synchronize()
            w = time.perf_counter() - t0
            if rep > 0:
                best = w if best is None else min(best, w)
        pf, pd = PAPER_TIMES["table3"][n]
        rows.append({"workload": "table3", "n": f"{n}x{n}", "eps": 0.01, "iterations": r.iterations,
                     "domain": "plain", "status": r.status, "w1": r.w1,
                     "marginal_err": r.marginal_err, "gpu_s": best, "paper_fs1_cpu_s": pf,
                     "paper_dense_cpu_s": pd, "speedup_vs_paper_fs1": pf / best})
        log(f"table3 {n}x{n}: {r.iterations} it, {best * 1e3:.2f} ms per solve "
            f"(paper's 2-D FS-1 on its CPU: {pf * 1e3:.1f} ms), w1 {r.w1:.12g}")
    return {"rows": rows,
            "note": "paper times: FS-1 and dense Sinkhorn on the paper's CPU (context, not a "
                    "target); GPU: one MI355X, binary64, fixed iteration counts, inputs "
                    "resident in HBM"}


def large_n_study(fs1, ctx, inputs, np, torch):
    """N = 1e8, eps = 1e-4, 2000 iterations, log domain: binary64 and binary32,
    with the CDF closed form of W1 for reference."""
    n = 100_000_000
    mu_np, nu_np = inputs.shifted_noisy_pair(n, 8, 3)
    w1_cdf = float(np.abs(np.cumsum(mu_np) - np.cumsum(nu_np)).sum() / n)
    mu = torch.tensor(mu_np, dtype=torch.float64, device="cuda")
    nu = torch.tensor(nu_np, dtype=torch.float64, device="cuda")
    del mu_np, nu_np
    rows = {}
    for dt in ("f64", "f32"):
        ctx.set_profiling(PROFILE_STRIDE)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fs1.fs1_solve(mu, nu, 1e-4, 0.0, itr_max=2000, dtype=dt, domain="log",
                          sync_every=64, ctx=ctx)
        torch.cuda.synchronize()
        w = time.perf_counter() - t0
        kms, kl, kb = ctx.kernel_stats()
        ctx.set_profiling(0)
        rows[dt] = {"iterations": r.iterations, "w1": r.w1, "marginal_err": r.marginal_err,
                    "s": round(w, 3), "grid_pts_it_per_s": n * r.iterations / w,
                    "kernel_GBps": kb / (kms * 1e-3) / 1e9 if kms else None,
                    "kernel_frac_hbm": (kb / (kms * 1e-3) / 1e9) / HBM_PEAK_GBS if kms else None}
        log(f"large N f{dt}: {r.iterations} it in {w:.2f} s, w1 {r.w1:.12g}, "
            f"err {r.marginal_err:.3e}, kernel {rows[dt]['kernel_GBps']:.0f} GB/s")
    rows["w1_cdf"] = w1_cdf
    rows["rel_w1_f32_vs_f64"] = abs(rows["f32"]["w1"] - rows["f64"]["w1"]) / rows["f64"]["w1"]
    rows["rel_w1_f64_vs_cdf"] = abs(rows["f64"]["w1"] - w1_cdf) / w1_cdf
    return rows


def batched_study(fs1, ctx, inputs, np, torch, B: int):
    """Uneven batch: B pairs, N log-uniform in [256, 65536], eps uniform over
    {1e-2, 3e-3, 1e-3}, 3-5 component mixtures, tol 1e-6 per instance,
    itr_max 5000.  The batched binary32 solve (one launch per half-iteration
    and run-length class, graph-replayed) is timed as solves/s and set beside
    the binary64 single-solve path (fs1_solve, log domain, one pair at a time)
    timed on a sample of the same instances."""
    seed = 2025
    spec = inputs.batch_spec(B, 256, 65536, [1e-2, 3e-3, 1e-3], seed)
    mu_np, nu_np, offs = inputs.batch_hists(spec)
    mu = torch.tensor(mu_np, dtype=torch.float64, device="cuda")
    nu = torch.tensor(nu_np, dtype=torch.float64, device="cuda")
    tol = [1e-6] * B
    log(f"batched: B={B}, sum N={int(offs[-1])}")

    def run(dt):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fs1.fs1_solve_batched(mu, nu, offs, spec.eps, tol, itr_max=5000, dtype=dt,
                                    sync_every=32, ctx=ctx)
        torch.cuda.synchronize()
        return res, time.perf_counter() - t0

    run("f32")  # warm-up (graph instantiation, workspace growth)
    rows = {}
    for dt in ("f32", "f64"):
        res, w = run(dt)
        its = np.array([r.iterations for r in res])
        ok = sum(r.status == 0 for r in res)
        conv = sum(r.converged for r in res)
        rows[dt] = {"s": round(w, 4), "solves_per_s": B / w, "converged": conv, "ok": ok,
                    "iterations_median": float(np.median(its)), "iterations_max": int(its.max()),
                    "grid_pts_it_per_s": float(np.sum(spec.sizes * its) / w),
                    "max_marginal_err_converged": max(
                        (r.marginal_err for r in res if r.converged), default=None)}
        log(f"batched {dt}: {w * 1e3:.1f} ms, {B / w:.1f} solves/s, {conv}/{B} converged, "
            f"iterations median {np.median(its):.0f} max {its.max()}")
        if dt == "f32":
            res32 = res
    # binary64 single-solve path on a sample of the same instances
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(B, size=min(64, B), replace=False))
    wsum = 0.0
    rel = []
    for i in sample:
        a, b = int(offs[i]), int(offs[i + 1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fs1.fs1_solve(mu[a:b].clone(), nu[a:b].clone(), float(spec.eps[i]), 1e-6,
                          itr_max=5000, dtype="f64", domain="log", sync_every=64, ctx=ctx)
        torch.cuda.synchronize()
        wsum += time.perf_counter() - t0
        if r.status == 0 and res32[i].status == 0:
            rel.append(abs(res32[i].w1 - r.w1) / abs(r.w1))
    single = len(sample) / wsum
    rows["single_f64"] = {"solves_per_s": single, "sample": int(len(sample)),
                          "note": "fs1_solve per pair (log domain, binary64, tol 1e-6); "
                                  "clone of each pair included in the timing"}
    rows["speedup_f32_batched_vs_f64_single"] = rows["f32"]["solves_per_s"] / single
    rows["max_rel_w1_f32_batched_vs_f64_single"] = max(rel) if rel else None
    rows["config"] = {"B": B, "n_lo": 256, "n_hi": 65536, "eps": [1e-2, 3e-3, 1e-3],
                      "tol": 1e-6, "itr_max": 5000, "seed": seed, "sum_n": int(offs[-1])}
    log(f"single f64 path: {single:.1f} solves/s on {len(sample)} sampled pairs; "
        f"batched f32 speedup {rows['speedup_f32_batched_vs_f64_single']:.1f}x")
    return rows


def serve_run(fs1, srv, pool, np, arrivals, window: float, drain: bool):
    """Feed `arrivals` (s, sorted) into the server in wall-clock time; requests
    cycle through the pool of device pairs.  Returns latencies (s) of the
    completed requests, completions inside the window and the elapsed time."""
    t_arr = {}
    lat = []
    done_in_window = 0
    k = 0
    t0 = time.perf_counter()
    while True:
        now = time.perf_counter() - t0
        while k < len(arrivals) and arrivals[k] <= now and now < window:
            m, v, e = pool[k % len(pool)]
            t_arr[srv.submit(m, v, e, 1e-6)] = arrivals[k]
            k += 1
        srv.step()
        now = time.perf_counter() - t0
        for t, r, a, c in srv.poll():
            lat.append(now - t_arr.pop(t))
            if now <= window:
                done_in_window += 1
            if r.status != 0:
                raise RuntimeError(f"request {t} failed: {r}")
        info = srv.info()
        if now >= window and (not drain or (info["queued"] == 0 and info["active"] == 0)):
            return np.array(lat), done_in_window, now, info, k


def serving_study(fs1, ctx, inputs, np, torch, seconds: float):
    """Request stream: Poisson arrivals, each request a seeded mixture pair with
    N log-uniform in [128, 2^20] and eps in {1e-2, 1e-3}, tol 1e-6, binary32
    scans, 64 GB admission budget.  Requests cycle through a pool of 256
    distinct device-resident pairs.  Two runs: the offered 20k requests/s
    (saturating: solves/s is the server's capacity, latency includes the
    growing queue) and half of the measured capacity (latency at a sustainable
    rate, drained at the end)."""
    seed = 77
    P = 256
    spec = inputs.batch_spec(P, 128, 1 << 20, [1e-2, 1e-3], seed)
    mu_np, nu_np, offs = inputs.batch_hists(spec)
    pool = []
    for i in range(P):
        a, b = int(offs[i]), int(offs[i + 1])
        pool.append((torch.tensor(mu_np[a:b], dtype=torch.float64, device="cuda"),
                     torch.tensor(nu_np[a:b], dtype=torch.float64, device="cuda"),
                     float(spec.eps[i])))
    torch.cuda.synchronize()
    log(f"serving: pool of {P} pairs, mean N {offs[-1] / P:.0f}")
    srv = fs1.Server(hbm_budget=64 << 30, max_active=4096, dtype="f32", itr_max=10000,
                     iters_per_step=16, ctx=ctx)
    # warm-up: a few requests through the server
    for m, v, e in pool[:8]:
        srv.submit(m, v, e, 1e-6)
    while srv.info()["active"] or srv.info()["queued"]:
        srv.step()
        srv.poll()
    out = {}
    rate = 20000.0
    arr = inputs.poisson_arrivals(rate, seconds, seed)
    lat, nwin, el, info, sub = serve_run(fs1, srv, pool, np, arr, seconds, drain=False)
    cap = nwin / seconds
    out["offered_20k"] = {
        "offered_per_s": rate, "window_s": seconds, "submitted": int(sub),
        "completed_in_window": int(nwin), "solves_per_s": cap,
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
        "p99_latency_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
        "left_queued": int(info["queued"]), "left_active": int(info["active"]),
        "note": "offered load above capacity: latency includes a queue that grows "
                "through the window"}
    log(f"serving at 20k req/s offered: {cap:.1f} solves/s, p50 "
        f"{out['offered_20k']['p50_latency_ms']:.1f} ms p99 "
        f"{out['offered_20k']['p99_latency_ms']:.1f} ms, {info['queued']} still queued")
    srv.close()
    srv = fs1.Server(hbm_budget=64 << 30, max_active=4096, dtype="f32", itr_max=10000,
                     iters_per_step=16, ctx=ctx)
    rate2 = max(1.0, 0.5 * cap)
    arr = inputs.poisson_arrivals(rate2, seconds, seed + 1)
    lat, nwin, el, info, sub = serve_run(fs1, srv, pool, np, arr, seconds, drain=True)
    out["half_capacity"] = {
        "offered_per_s": rate2, "window_s": seconds, "submitted": int(sub),
        "completed": int(lat.size), "solves_per_s": lat.size / el,
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
        "p99_latency_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None}
    log(f"serving at {rate2:.0f} req/s: p50 {out['half_capacity']['p50_latency_ms']:.1f} ms "
        f"p99 {out['half_capacity']['p99_latency_ms']:.1f} ms")
    srv.close()
    out["config"] = {"pool": P, "n_lo": 128, "n_hi": 1 << 20, "eps": [1e-2, 1e-3], "tol": 1e-6,
                     "hbm_budget_bytes": 64 << 30, "dtype": "f32", "iters_per_step": 16,
                     "seed": seed}
    return out


if __name__ == "__main__":
    main()
