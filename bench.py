#!/usr/bin/env python3
"""Throughput of one PISO step of the micro-continuum DBS method on one MI355X.

Workload: the 256^3 fractured porous matrix (log-normal permeability, mean
log10 k = -13, sigma 0.5, 8-cell correlation; porosity U[0.2, 0.4]; three
random planar fractures 8 cells wide; water displacing oil), in the mixed
precision form (FP32 multigrid inside FP64 CG, FP64 MULES), pressure solved
to a relative residual of 1e-8.  The same workload in plain FP64 at the same
tolerance is timed beside it (equal final accuracy).

Metric: cell-updates/s = cells / wall time of one full step (alpha transport,
momentum predictor, two pressure correctors), inputs resident in HBM.

Also reported: the roofline fraction of the dominant kernel, measured live
with HIP events on the library stream over the timed region, and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD public figure


def alg_bytes_per_cell(cls: str, rsize: int) -> float:
    """Algorithmic bytes per fine cell and launch of a kernel class.

    rsize = 8 (FP64 V-cycle) or 4 (FP32 V-cycle).  Red-black half sweeps touch
    every coefficient (rAU) once, half of b, the other colour of x and write
    their own colour of x.
    """
    s = rsize
    return {
        # rAU (all), b (own colour), x (other colour) read; own colour written
        "smooth_fine": s + 0.5 * s + 0.5 * s + 0.5 * s,
        # zero initial guess: rAU and own-colour b read, both colours written
        "smooth_fine_zero": s + 0.5 * s + s,
        # prolongation fused in the first up-sweep: x and the coarse
        # correction read, rAU and own-colour b read, both colours written
        "prolong_fine": s + s / 8.0 + s + 0.5 * s + s,
        # red residuals only: x and rAU read, red b read, coarse b written
        "restrict_fine": 2 * s + 0.5 * s + s / 8.0,
        "spmv": 24.0,                  # rAU, p read; q written (FP64)
        "axpy": 48.0,                  # x, p, r, q read; x, r written
        "dot": 8.0 + s + (s if s == 4 else 0.0),
        "xpby": 8.0 + s + 8.0 + (s if s == 4 else 0.0),
    }.get(cls, 0.0)


def measured_traffic(kernel, precision, n):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summaries (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter's
    reading for a plain copy of known size).  None when no summary matches
    this kernel, precision and size, or when the kernel source has changed
    since the counters were taken."""
    import glob
    import hashlib
    import re
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        m = re.search(r"<!-- bench-traffic (\{.*?\}) -->", open(path).read())
        if not m:
            continue
        rec = json.loads(m.group(1))
        if (rec.get("kernel"), rec.get("precision"), rec.get("n")) != (kernel, precision, n):
            continue
        src = os.path.join(ROOT, rec["source"])
        if not os.path.exists(src):
            continue
        if hashlib.sha1(open(src, "rb").read()).hexdigest() != rec["source_sha1"]:
            continue
        return float(rec["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


def time_solver(case, precision, steps, warmup, prof_class=None, profile_all=False):
    import torch
    from paper_2003_08374_amd import dbs

    s = dbs.Solver(case, precision=precision)
    s.step(warmup)
    all_times = None
    if profile_all:
        s.set_profiling((1 << 62) - 1)
        s.reset_profiling()
        s.step(1)
        all_times = s.kernel_times()
        s.set_profiling(0)
    dom = prof_class
    if dom is None and all_times:
        dom = max(all_times.items(), key=lambda kv: kv[1][1])[0]
    if dom:
        s.set_profiling(1 << dbs.Solver.kernel_class(dom))
    s.reset_profiling()
    its = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.step(1)
        its.append(s.stats()["p_iters"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = s.kernel_times()
    st = s.stats()
    s.close()
    return {"sec": t1 - t0, "p_iters": its, "kernel": dom, "ktimes": kt, "all": all_times,
            "stats": st}


def cpu_baseline(n=64, steps=2):
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O
    from paper_2003_08374_amd import workloads as W

    O.build(force=False)
    c = W.fractured_3d(n=n, seed_k=3, seed_phi=4, fractures="planes", frac_seed=5,
                       n_frac=3).replace(p_tol=1e-8)
    st = O.initial_state(c)
    t0 = time.perf_counter()
    O.step(c, st, steps)
    dt = time.perf_counter() - t0
    return {
        "value": n ** 3 * steps / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
        "sample": (f"{n}^3 instance of the same generator (k seed 3, phi seed 4, 3 planar "
                   f"fractures), {steps} steps from rest, p_tol 1e-8, single thread; the "
                   f"oracle's Jacobi-CG cost per cell grows with n, so this sample "
                   f"flatters the CPU"),
        "seconds": dt,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--p-tol", type=float, default=1e-8)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--kernel", default=None, help="kernel class for the roofline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}): the "
              "multi-GPU decomposition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain copy of known size: 2^27 doubles = 1 GiB read + 1 GiB written
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 8, "launches": 3}))
        return
    from paper_2003_08374_amd import workloads as W

    case = W.fractured_3d(n=args.n, seed_k=3, seed_phi=4, fractures="planes", frac_seed=5,
                          n_frac=3, name=f"fractured_3d_{args.n}_planes")
    case = case.replace(p_tol=args.p_tol, p_maxit=500)
    cells = case.ncells

    main_run = time_solver(case, args.precision, args.steps, args.warmup,
                           prof_class=args.kernel, profile_all=args.kernel is None)
    ms = main_run["sec"] / args.steps * 1e3
    value = cells / (main_run["sec"] / args.steps)
    rsize = 4 if args.precision == "mixed" else 8
    kname = main_run["kernel"]
    launches, kms = main_run["ktimes"].get(kname, (0, 0.0))
    per_cell = alg_bytes_per_cell(kname, rsize)
    roof = None
    if launches and per_cell:
        avg_s = kms / launches * 1e-3
        achieved = per_cell * cells / avg_s / 1e9
        traffic, tsrc = measured_traffic(kname, args.precision, args.n)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "kernel": kname, "alg_bytes_per_launch": per_cell * cells,
                "avg_launch_us": round(avg_s * 1e6, 2), "launches": launches}
        if traffic:
            roof["traffic_rate_GBs"] = round(traffic / avg_s / 1e9, 1)
            roof["traffic_source"] = tsrc

    fp64 = None
    if not args.no_fp64 and args.precision == "mixed":
        r64 = time_solver(case, "fp64", args.steps, args.warmup, prof_class=kname)
        fp64 = {"value": cells / (r64["sec"] / args.steps),
                "ms_per_step": r64["sec"] / args.steps * 1e3,
                "p_iters_last": r64["p_iters"][-1]}
    cpu = None if args.no_cpu else cpu_baseline()

    # whole-step bytes from the profile of all kernel classes (ideal model)
    line = {
        "metric": "cell-updates/s per PISO step at 256^3 (FP64 vs mixed/batched); % HBM roofline",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": case.name, "cells": cells, "precision": args.precision,
                   "p_tol": args.p_tol, "n_corr": case.n_corr, "dt": case.dt,
                   "p_iters_last_step": main_run["p_iters"][-1]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64_same_tol": fp64,
        "speedup_mixed_vs_fp64": (value / fp64["value"]) if fp64 else None,
    }
    if main_run["all"]:
        line["kernel_ms_one_step"] = {k: round(v[1], 3) for k, v in sorted(
            main_run["all"].items(), key=lambda kv: -kv[1][1])}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
