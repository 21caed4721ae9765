"""The project's tuner of the batched solve's per-instance configuration.

For every dtype and every half-octave class of grid sizes n (129 ... 2^20) it
times each configuration the batched kernels are built for -- the shared
chunk launches with run length R, and the resident form (one workgroup of nt
threads per instance, all iterations in one launch) where the instance fits
-- on a batch of equal-size seeded mixture pairs (about 2^24 grid points in
all, eps = 1e-2, 100 iterations, tol 0), through fs1_solve_batched_config.
The fastest resident form and the fastest shared run length of each class
become a row of csrc/fs1_tune_table.h, which fs1_solve_batched and the server
read (fs1_tune.h).  A class keeps the built-in rule's choice unless another
candidate is at least 3% faster, so timing noise does not flip it.

Usage (on the target GPU):  python -m paper_2202_10042_amd.tune [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(PKG, "csrc", "fs1_tune_table.h")

SHARED_R = {"f64": (8,), "f32": (16, 8, 4)}
RESIDENT = {"f64": ((8, 256), (8, 1024)),
            "f32": ((16, 256), (8, 256), (8, 1024), (4, 256), (4, 1024))}
KEEP_MARGIN = 0.03


def classes():
    """Half-octave classes (n_lo, n_max] from 128 to 2^20."""
    edges = [128] + [int(round(2.0 ** (k / 2.0))) for k in range(15, 41)]
    return list(zip(edges[:-1], edges[1:]))


def rule_config(dtype: str, n: int):
    """The built-in rule at eps = 1e-2 (h/eps small): resident in one
    workgroup when it fits (256 threads x 16 / 8, else 1024 x 8), else the
    longest run length."""
    rmax = 16 if dtype == "f32" else 8
    if n <= 256 * rmax:
        return (rmax, 256)
    if n <= 1024 * 8:
        return (8, 1024)
    return (rmax, 0)


def time_config(fs1, torch, mu, nu, offs, eps, dtype, cfg, iters):
    B = len(offs) - 1
    tol = [0.0] * B
    fs1.fs1_solve_batched(mu, nu, offs, eps, tol, itr_max=10, dtype=dtype, config=cfg)
    best = None
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fs1.fs1_solve_batched(mu, nu, offs, eps, tol, itr_max=iters, dtype=dtype,
                                    config=cfg)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if any(r.status != 0 for r in res):
            raise RuntimeError(f"config {cfg} failed")
        best = dt if best is None else min(best, dt)
    return best


def tune(points: int = 1 << 24, iters: int = 100, log=print):
    import numpy as np
    import torch

    from . import fs1, inputs
    rows = []
    for dtype in ("f64", "f32"):
        for lo, hi in classes():
            n = int(round(math.sqrt(lo * hi)))
            m = max(8, min(4096, points // n))
            seeds = 5000 + 2 * np.arange(m)
            mu, nu, offs = inputs.mixture_pairs_device([n] * m, [3] * m, seeds, torch)
            eps = [1e-2] * m
            cands = [(r, 0) for r in SHARED_R[dtype]]
            cands += [(r, nt) for r, nt in RESIDENT[dtype] if n <= r * nt]
            times = {}
            for cfg in cands:
                times[cfg] = time_config(fs1, torch, mu, nu, offs, eps, dtype, cfg, iters)
            rule = rule_config(dtype, n)
            per = lambda c: times[c] / (m * iters) * 1e6  # us per instance-iteration
            best = min(times, key=times.get)
            if rule in times and times[best] > (1.0 - KEEP_MARGIN) * times[rule]:
                best = rule
            shared = [c for c in times if c[1] == 0]
            best_sh = min(shared, key=times.get)
            rule_sh = (16 if dtype == "f32" else 8, 0)
            if times[best_sh] > (1.0 - KEEP_MARGIN) * times[rule_sh]:
                best_sh = rule_sh
            rows.append({"dtype": dtype, "n_lo": lo, "n_max": hi, "n": n, "instances": m,
                         "best": best, "best_shared": best_sh, "rule": rule,
                         "us_per_instance_iteration": {f"{r}x{nt}": round(per((r, nt)), 4)
                                                       for r, nt in times}})
            log(f"{dtype} n in ({lo}, {hi}] (n={n}, {m} instances): best {best} "
                f"({per(best):.3f} us), shared {best_sh}, rule {rule} "
                f"({per(rule) if rule in times else float('nan'):.3f} us)")
            del mu, nu
            torch.cuda.empty_cache()
    return rows


def write_table(rows, path: str = TABLE, device: str = ""):
    lines = [
        "// fs1_tune_table.h -- measured per-class configurations of the batched solve",
        "// (see fs1_tune.h), written by paper_2202_10042_amd/tune.py from timings of",
        f"// forced configurations{(' on ' + device) if device else ''}: per class, the fastest",
        "// resident form (R_res, nt; nt = 0 when the shared launches are faster) and",
        "// the fastest shared run length, each kept at the built-in rule's choice",
        "// unless another candidate is at least 3% faster.  Columns: dtype (0",
        "// binary64, 1 binary32), the class's largest n, R_shared, R_res, nt; the",
        "// comment gives the time per instance-iteration of the chosen form.",
        "#pragma once",
        "",
        "namespace fs1 {",
        "",
        "struct TuneRow {",
        "  int dtype;        // 0 binary64, 1 binary32",
        "  long long n_max;  // the row covers n <= n_max (rows ascend within a dtype)",
        "  int R_shared;     // fastest run length in the shared launches",
        "  int R_res;        // fastest resident configuration (R_res, nt), nt = 0: none faster",
        "  int nt;",
        "};",
        "",
        "static const TuneRow kTuneRows[] = {",
    ]
    for r in rows:
        dt = 0 if r["dtype"] == "f64" else 1
        (rb, ntb) = r["best"]
        rs = r["best_shared"][0]
        us = r["us_per_instance_iteration"][f"{rb}x{ntb}"]
        lines.append(f"    {{{dt}, {r['n_max']}, {rs}, {rb if ntb else 0}, {ntb}}},  "
                     f"// n ~ {r['n']}: {us} us")
    lines += ["};", "", "}  // namespace fs1", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--json", default=None, help="also write the timings here")
    ap.add_argument("--iters", type=int, default=100)
    args = ap.parse_args()
    import torch
    rows = tune(iters=args.iters, log=lambda *a: print(*a, file=sys.stderr, flush=True))
    name = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else ""
    write_table(rows, args.out, name)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(rows, f, indent=1)
    print(args.out)


if __name__ == "__main__":
    main()
