"""The project's tuner of the batched solve's per-instance configuration.

Stage 1 (per class): for every dtype and every half-octave class of grid
sizes n (129 ... 2^20) it times each configuration the batched kernels are
built for -- the shared chunk launches with run length R, and the resident
form (one workgroup of nt threads per instance, all iterations in one launch)
where the instance fits -- on a batch of equal-size seeded mixture pairs
(about 2^24 grid points in all, eps = 1e-2, 100 iterations, tol 0), through
fs1_solve_batched_config.  The fastest resident form and the fastest shared
run length of each class form a row.

Stage 2 (the mix): in an uneven batch, instances of different run lengths
need separate shared launches, and resident workgroups hold their wave slots
for all their iterations, competing with the shared launches of the larger
instances -- effects no equal-size batch shows.  On an uneven batch of the
batched path's own kind (4096 pairs, N log-uniform in [256, 65536], eps
uniform over {1e-2, 3e-3, 1e-3}, tol 1e-6, itr_max 5000; a seed other than
the benchmark's) it times, per dtype, the stage-1 shared run lengths against
the rule's for every class, then the resident form cut off above each class
edge, and keeps the fastest.

A choice replaces the built-in rule only when it is at least 3% faster in
stage 1 (per-class timings of 100 iterations) and 1.5% faster in stage 2
(whole batches), so timing noise does not flip it.
The rows become csrc/fs1_tune_table.h, which fs1_solve_batched and the server
read (fs1_tune.h).

Usage (on the target GPU):
  python -m paper_2202_10042_amd.tune [--out PATH] [--json PATH]
  python -m paper_2202_10042_amd.tune --stage1-json OLD.json   (stage 2 only)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(PKG, "csrc", "fs1_tune_table.h")

SHARED_R = {"f64": (8,), "f32": (16, 8, 4)}
RESIDENT = {"f64": ((8, 256), (8, 1024)),
            "f32": ((16, 256), (8, 256), (8, 1024), (4, 256), (4, 1024))}
KEEP_MARGIN = 0.03
# stage 2 times whole batches of about a second, whose repeat-to-repeat noise is
# a few tenths of a percent (two identical configurations measured 0.3% apart)
MIX_MARGIN = 0.015


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


def read_table(path: str = TABLE):
    """Rows of a written table, in the form tune() returns them (timings left
    out; the comment of each row is kept)."""
    rows = []
    prev = {}
    pat = re.compile(r"\{(\d), (\d+), (\d+), (\d+), (\d+)\},\s*//\s*(.*)")
    for m in pat.finditer(open(path).read()):
        dt, nmax, rs, rr, nt = (int(v) for v in m.groups()[:5])
        dtype = "f64" if dt == 0 else "f32"
        lo = prev.get(dtype, 128)
        prev[dtype] = nmax
        rows.append({"dtype": dtype, "n_lo": lo, "n_max": nmax, "best_shared": (rs, 0),
                     "best": (rr, nt) if nt else (rs, 0), "comment": m.group(6)})
    return rows


def run_length_bound(dtype: str, c: float) -> int:
    """The longest run the batched kernels allow at c = h/eps (the library's
    pick_run_length for the log domain)."""
    if dtype == "f64":
        return 8 if 7.0 * c <= 600.0 else 1
    for r in (16, 8, 4):
        if (r - 1) * c <= 60.0:
            return r
    return 1


def instance_config(rows, dtype: str, n: int, eps: float, cut=None):
    """(R, nt) of an instance under the rows (as the library's batch_config),
    with the resident form cut off above n = cut."""
    rmax = run_length_bound(dtype, (1.0 / n) / eps)
    row = next(r for r in rows if r["dtype"] == dtype and n <= r["n_max"])
    rr, nt = row["best"]
    if nt and rr <= rmax and n <= rr * nt and (cut is None or n <= cut):
        return (rr, nt)
    r = min(row["best_shared"][0], rmax)
    while r > 1 and r not in ((8,) if dtype == "f64" else (16, 8, 4)):
        r //= 2
    return (r, 0)


def uniform_shared(rows, dtype: str):
    """The rows of one dtype with every shared run length at the built-in
    rule's (16 in binary32, 8 in binary64)."""
    rule = 16 if dtype == "f32" else 8
    out = []
    for r in rows:
        if r["dtype"] == dtype:
            r = dict(r, best_shared=(rule, 0))
            if r["best"][1] == 0:
                r["best"] = (rule, 0)
        out.append(r)
    return out


def mix_stage(rows, reps: int = 3, log=print, seed: int = 77):
    """Stage 2 on an uneven batch, per dtype: (a) the shared run length, per
    class as stage 1 found it or the rule's for every class (instances of
    different run lengths need separate launches, whose latency stage 1 does
    not see); (b) then the resident cut-off.  Returns the rows and the
    timings."""
    import numpy as np
    import torch

    from . import fs1, inputs
    B = 4096
    spec = inputs.batch_spec(B, 256, 65536, [1e-2, 3e-3, 1e-3], seed)
    mu_np, nu_np, offs = inputs.batch_hists(spec)
    mu = torch.tensor(mu_np, dtype=torch.float64, device="cuda")
    nu = torch.tensor(nu_np, dtype=torch.float64, device="cuda")
    sizes = np.diff(np.asarray(offs)).astype(int)
    tol = [1e-6] * B

    def timed(dtype, rws, cut):
        cfg = [instance_config(rws, dtype, int(n), float(e), cut)
               for n, e in zip(sizes, spec.eps)]
        fs1.fs1_solve_batched(mu, nu, offs, spec.eps, tol, itr_max=5000, dtype=dtype,
                              sync_every=32, config=cfg)
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fs1.fs1_solve_batched(mu, nu, offs, spec.eps, tol, itr_max=5000, dtype=dtype,
                                  sync_every=32, config=cfg)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best

    timings = {}
    for dtype in ("f64", "f32"):
        uni = uniform_shared(rows, dtype)
        t_rows, t_uni = timed(dtype, rows, None), timed(dtype, uni, None)
        log(f"mix {dtype}: shared run lengths per class {t_rows * 1e3:.1f} ms, "
            f"the rule's for every class {t_uni * 1e3:.1f} ms")
        if t_rows > (1.0 - MIX_MARGIN) * t_uni:
            rows = uni
        edges = sorted({r["n_max"] for r in rows if r["dtype"] == dtype and r["best"][1]})
        times = {None: t_uni if rows is uni else t_rows}
        for cut in edges[:-1] + [0]:
            times[cut] = timed(dtype, rows, cut)
            log(f"mix {dtype}: resident up to n = {cut}: {times[cut] * 1e3:.1f} ms")
        pick = min(times, key=times.get)
        if times[pick] > (1.0 - MIX_MARGIN) * times[None]:
            pick = None
        log(f"mix {dtype}: resident cut-off {pick}")
        rows = apply_cuts(rows, {dtype: pick})
        timings[dtype] = {"shared_per_class_ms": round(t_rows * 1e3, 2),
                          "shared_rule_ms": round(t_uni * 1e3, 2),
                          "cut_ms": {str(k): round(v * 1e3, 2) for k, v in times.items()},
                          "cut": pick}
    return rows, timings


def apply_cuts(rows, cuts):
    """Rows with the resident form removed above each dtype's cut-off."""
    out = []
    for r in rows:
        r = dict(r)
        cut = cuts.get(r["dtype"])
        if cut is not None and r["best"][1] and r["n_max"] > cut:
            r["best"] = r["best_shared"]
            r["cut"] = cut
        out.append(r)
    return out


def write_table(rows, path: str = TABLE, device: str = ""):
    lines = [
        "// fs1_tune_table.h -- measured per-class configurations of the batched solve",
        "// (see fs1_tune.h), written by paper_2202_10042_amd/tune.py from timings of",
        f"// forced configurations{(' on ' + device) if device else ''}: per class, the fastest",
        "// resident form (R_res, nt; nt = 0 when the shared launches are faster) and",
        "// the fastest shared run length, each kept at the built-in rule's choice",
        "// unless another candidate is at least 3% faster; then, per dtype, on an",
        "// uneven batch (tune.py, stage 2), the shared run lengths per class or the",
        "// rule's for every class, and the resident form cut off above the class",
        "// edge that made the batch fastest, each kept unless 1.5% faster.",
        "// Columns: dtype (0 binary64, 1 binary32), the",
        "// class's largest n, R_shared, R_res, nt; the comment gives the row form's",
        "// time per instance-iteration in stage 1.",
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
        if "us_per_instance_iteration" in r:
            us = r["us_per_instance_iteration"].get(f"{rb}x{ntb}")
            note = f"n ~ {r['n']}: {us} us"
        else:
            note = r.get("comment", "").split(";")[0]
        if "cut" in r:
            note += f"; resident cut off above n = {r['cut']} (uneven batch)"
        lines.append(f"    {{{dt}, {r['n_max']}, {rs}, {rb if ntb else 0}, {ntb}}},  // {note}")
    lines += ["};", "", "}  // namespace fs1", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--json", default=None, help="also write the timings here")
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--stage1-json", default=None,
                    help="take the stage-1 rows from this earlier --json output and run "
                         "stage 2 only")
    args = ap.parse_args()
    import torch
    say = lambda *a: print(*a, file=sys.stderr, flush=True)
    if args.stage1_json:
        with open(args.stage1_json) as f:
            rows = json.load(f)["rows"]
        for r in rows:
            r["best"], r["best_shared"] = tuple(r["best"]), tuple(r["best_shared"])
    else:
        rows = tune(iters=args.iters, log=say)
    final, mix_t = mix_stage(rows, log=say)
    name = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] \
        if torch.cuda.is_available() else ""
    write_table(final, args.out, name)
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"rows": rows, "mix": mix_t}, f, indent=1)
    print(args.out)


if __name__ == "__main__":
    main()
