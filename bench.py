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

# Algorithmic bytes per cell of one PISO step, stage by stage (FP64 fields of
# 8 B; the ideal traffic of each stage with the fusion the model states):
# alpha face fluxes (alpha, 3 fluxes, phi, k^-1, p_rgh read; 3 antidiffusive
# fluxes and R+- written), MULES limit and update (alpha, 3 A, R+-, 3 F, phi
# read; alpha' and 3 limited fluxes written), momentum assembly (16 fields
# read, a_P and 3 sources written), one Jacobi sweep (15 read, 3 written),
# per corrector the p_rgh assembly (15 read, 8 written) and the flux and
# velocity correction (10 read, 6 written), and per PCG iteration the SpMV,
# the x/r update, the V-cycle (fine level with fused red-black sweeps, 8/7
# for the coarse levels) and the direction update: 216 B in FP64, about 160 B
# with the V-cycle in FP32.  The pressure initial guesses: the first
# corrector's extrapolation in time (p_rgh and its four previous values
# read and written, and per later corrector its three stored changes read),
# each later corrector's guess (p_rgh and the three stored changes read,
# p_rgh and its copy written) and the record of its change (p_rgh, the copy
# and the three stored changes read, the three changes written).
STEP_BYTES = {"alpha_face": 96, "alpha_limit_update": 112, "mom_assemble": 144,
              "jacobi_sweep": 144, "p_assembly": 184, "correct": 128,
              "guess_first": 80, "guess_later": 136,
              "pcg_iteration": {"fp64": 216, "mixed": 160}}


def alg_step_bytes_per_cell(precision, p_iters, sweeps, n_sub=1):
    """Algorithmic bytes per cell of one step with the measured PCG
    iterations per corrector and predictor sweeps (n_sub saturation
    sub-cycles repeat the transport stages)."""
    B = STEP_BYTES
    return (n_sub * (B["alpha_face"] + B["alpha_limit_update"]) + B["mom_assemble"] +
            sweeps * B["jacobi_sweep"] + len(p_iters) * (B["p_assembly"] + B["correct"]) +
            B["guess_first"] + (len(p_iters) - 1) * B["guess_later"] +
            sum(p_iters) * B["pcg_iteration"][precision])


def alg_bytes_per_cell(cls: str, rsize: int, fused: bool = False) -> float:
    """Algorithmic bytes per fine cell and launch of a kernel class.

    rsize = 8 (FP64 V-cycle) or 4 (FP32 V-cycle).  fused: the fine-level
    smoother launches are full red-black sweeps; else half sweeps, which
    read all of rAU, b on their own colour and x on the other colour, and
    write their own colour.
    """
    s = rsize
    if not fused and cls in ("smooth_fine", "smooth_fine_zero", "prolong_fine"):
        return {"smooth_fine": 2.5 * s,
                "smooth_fine_zero": s + 0.5 * s + s,
                "prolong_fine": s + s / 8.0 + s + 0.5 * s + s}[cls]
    return {
        # fused red-black sweep (both colours): x, b, rAU read once, x written
        "smooth_fine": 4 * s,
        # the last sweep of a mixed-precision V-cycle: z_old read as well
        # (b.z and b.z_old formed in the sweep)
        "smooth_fine_dot": 5 * s,
        # zero initial guess: b and rAU read, x written
        "smooth_fine_zero": 3 * s,
        # prolongation fused in the first up-sweep: x and the coarse
        # correction (one value per 8 cells) read as well
        "prolong_fine": 4 * s + s / 8.0,
        # red residuals only: x and rAU read, red b read, coarse b written
        "restrict_fine": 2 * s + 0.5 * s + s / 8.0,
        # direction update fused in: z (s), old p and rAU read; new p and q
        # written (FP64); in flexible (mixed) CG with half sweeps also a
        # copy z_old (s) (fused sweeps rotate three z buffers instead)
        "spmv": 32.0 + s + (s if s == 4 and not fused else 0.0),
        # true residual r = b - A x: x, rAU, b read; r (and its FP32 copy) written
        "residual": 32.0 + (4.0 if s == 4 else 0.0),
        # x, p, r, q read; x, r (and the FP32 copy of r) written
        "axpy": 48.0 + (4.0 if s == 4 else 0.0),
        # r (FP64) and z read, and z_old in flexible CG with half sweeps
        "dot": 8.0 + s + (s if s == 4 else 0.0),
        # clear-fluid CSF, both launches of a step: Gauss gradient of alpha
        # (alpha read, 3 components written) and curvature (gradients, phi,
        # k^-1 read, sigma kappa / phi written)
        "curvature": 32.0 + 48.0,
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
        for m in re.finditer(r"<!-- bench-traffic (\{.*?\}) -->", open(path).read()):
            rec = json.loads(m.group(1))
            if (rec.get("kernel"), rec.get("precision"), rec.get("n")) != (kernel, precision, n):
                continue
            if "sources" not in rec or sources_sha1(rec["sources"]) != rec.get("sources_sha1"):
                continue
            return float(rec["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


CSRC = ["paper_2003_08374_amd/csrc/" + f for f in
        ("api.hip", "k_alpha.hip", "k_momentum.hip", "k_pressure.hip", "dbs_device.h",
         "dbs_internal.h")]


def sources_sha1(files):
    """One SHA-1 over the named source files (repository-relative)."""
    import hashlib
    h = hashlib.sha1()
    for f in files:
        path = os.path.join(ROOT, f)
        if not os.path.exists(path):
            return None
        h.update(open(path, "rb").read())
    return h.hexdigest()


def summarize_counters(d, n, precision, cmd_trace, cmd_counters):
    """Markdown summary of a whole-step rocprofv3 measurement of the 256^3
    workload: a kernel trace (d/trace), FETCH_SIZE and WRITE_SIZE passes
    (d/fetch, d/write) and the same passes over a plain 1 GiB copy
    (d/cfetch, d/cwrite) for the calibration.  The timed call of each run
    (its last dbs_step call, several steps) is summarised per step, the same
    steps whose time the benchmark reports."""
    import csv
    import re

    def rows(p):
        with open(p) as f:
            return list(csv.DictReader(f))

    def name(x):
        return re.sub(r"\(.*$", "", x["Kernel_Name"]).replace("void ", "").replace("dbs::", "")

    def timed_call(rs):
        # the last dbs_step call: from the end of the call before it (its
        # k_stats_final) to the end of this one; k_add_time marks each step
        key = "Dispatch_Id" if "Dispatch_Id" in rs[0] else "Start_Timestamp"
        rs = sorted(rs, key=lambda x: int(x[key]))
        adds = [i for i, x in enumerate(rs) if name(x) == "k_add_time"]
        fins = [i for i, x in enumerate(rs) if name(x) == "k_stats_final"]
        last = adds[-1]
        end = min([i for i in fins if i > last], default=len(rs) - 1)
        start = max([i for i in fins if i < last], default=-1) + 1
        seg = rs[start:end + 1]
        return seg, sum(1 for x in seg if name(x) == "k_add_time")

    def calib(kind):
        v = [float(x["Counter_Value"]) for x in rows(f"{d}/c{kind}/run_counter_collection.csv")
             if "copyBuffer" in x["Kernel_Name"]]
        return (1 << 30) / 1024.0 / max(v)

    cf, cw = calib("fetch"), calib("write")
    cells = n ** 3
    tr, steps = timed_call(rows(f"{d}/trace/run_kernel_trace.csv"))
    fe, _ = timed_call(rows(f"{d}/fetch/run_counter_collection.csv"))
    wr, _ = timed_call(rows(f"{d}/write/run_counter_collection.csv"))
    agg = {}
    def grid(x):  # threads in the launch (the two files name the field differently)
        if "Grid_Size" in x:
            return int(x["Grid_Size"])
        return int(x["Grid_Size_X"]) * int(x["Grid_Size_Y"]) * int(x["Grid_Size_Z"])

    for x in tr:
        k = (name(x), grid(x))
        a = agg.setdefault(k, {"n": 0, "us": 0.0, "f": 0.0, "w": 0.0, "nc": 0})
        a["n"] += 1
        a["us"] += (int(x["End_Timestamp"]) - int(x["Start_Timestamp"])) * 1e-3
    for src, key, fac in ((fe, "f", cf), (wr, "w", cw)):
        cnt = {}
        for x in src:
            k = (name(x), grid(x))
            if k in agg:
                agg[k][key] += float(x["Counter_Value"]) * 1024.0 * fac
                cnt[k] = cnt.get(k, 0) + 1
        for k, c in cnt.items():
            agg[k][key] /= c  # bytes per launch
    # per step of the timed call
    for a in agg.values():
        a["n"] /= steps
        a["us"] /= steps
    span = (max(int(x["End_Timestamp"]) for x in tr) - int(tr[0]["Start_Timestamp"])) * 1e-6
    span /= steps
    busy = sum(a["us"] for a in agg.values()) * 1e-3
    step_bytes = sum((a["f"] + a["w"]) * a["n"] for a in agg.values())
    lines = [f"# One PISO step, {n}^3 fractured workload, {precision}: kernel times and HBM "
             "traffic", "",
             "Commands (from /tmp, `export TMPDIR=/tmp`; `<out>` is the output folder):", "",
             "```", cmd_trace, cmd_counters, "```", "",
             f"Calibration: a plain 1 GiB device copy reads FETCH_SIZE x {cf:.4f} and "
             f"WRITE_SIZE x {cw:.4f} of the bytes it moves.", "",
             f"Per step of the timed call of the trace run ({steps} steps, the ones the "
             f"benchmark times): {len(tr) / steps:.1f} launches, kernel time {busy:.3f} ms over "
             f"a span of {span:.3f} ms (the tracer adds a few us per launch).  Counted HBM "
             f"traffic per step: {step_bytes / 1e9:.2f} GB = "
             f"{step_bytes / cells:.0f} B per cell.", "",
             "| kernel | threads | launches per step | avg us | ms per step | MB per launch | "
             "B per cell | GB/s |", "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for (k, g), a in sorted(agg.items(), key=lambda kv: -kv[1]["us"]):
        if a["us"] < 1.0:
            continue
        avg = a["us"] / a["n"]
        mb = (a["f"] + a["w"]) / 1e6
        lines.append(f"| `{k}` | {g} | {a['n']:.1f} | {avg:.1f} | {a['us'] / 1e3:.3f} | {mb:.1f} | "
                     f"{(a['f'] + a['w']) / cells:.1f} | {(a['f'] + a['w']) / (avg * 1e-6) / 1e9:.0f} |")
    ax = [a for (k, g), a in agg.items() if k == "k_axpy_dot"]
    recs = [{"kernel": "step", "precision": precision, "n": n,
             "traffic_bytes_per_launch": step_bytes, "sources": CSRC,
             "sources_sha1": sources_sha1(CSRC)}]
    if ax:
        recs.append({"kernel": "axpy", "precision": precision, "n": n,
                     "traffic_bytes_per_launch": ax[0]["f"] + ax[0]["w"], "sources": CSRC,
                     "sources_sha1": sources_sha1(CSRC)})
    lines.append("")
    for r in recs:
        lines.append(f"<!-- bench-traffic {json.dumps(r)} -->")
    return "\n".join(lines) + "\n"


def step_roofline(run, cells, precision, ms, n):
    """Whole-step figures: the algorithmic bytes of the stage model with the
    last timed step's PCG iterations and predictor sweeps, over the measured
    step time; and, when a committed counter summary of this workload and
    source exists, the counted HBM bytes of one step over the same time."""
    its, sw = run["p_iters"][-1], run["sweeps"][-1]
    b_cell = alg_step_bytes_per_cell(precision, its, sw)
    t = ms * 1e-3
    out = {"alg_bytes_per_cell": b_cell, "p_iters": its, "predictor_sweeps": sw,
           "alg_GBs": round(b_cell * cells / t / 1e9, 1),
           "frac_alg": round(b_cell * cells / t / 1e9 / HBM_PEAK_GBS, 4)}
    counted, src = measured_traffic("step", precision, n)
    out["counter_bytes_per_step"] = counted
    out["frac_counters"] = (round(counted / t / 1e9 / HBM_PEAK_GBS, 4) if counted else None)
    if counted:
        out["counter_source"] = src
    return out


def class_table(run, cells, precision, n, its, mgc):
    """Per kernel class over one profiled step: milliseconds, and for the
    classes with a byte model the algorithmic rate and fraction of peak.
    The coarse multigrid sweeps (FP32, stored coefficients) read x, b, the
    three face coefficients and the diagonal and write x (28 B per coarse
    cell and sweep); at 256^3 the levels 128^3, 64^3 and 32^3 are cycled by
    grid kernels, 2 mgc sweeps each per V-cycle, one V-cycle per PCG
    iteration."""
    allt = run.get("all") or {}
    rs = 4 if precision == "mixed" else 8
    out = {}
    for k, (launches, kms) in sorted(allt.items(), key=lambda kv: -kv[1][1]):
        e = {"ms": round(kms, 3), "launches": launches}
        b = alg_bytes_per_cell(k, rs, True) * cells * launches
        if k == "residual":
            # the true residual is launched every iteration but works only
            # where it is wanted: the initial residual and the confirming
            # check of each solve (the other launches exit at once)
            b = alg_bytes_per_cell(k, rs, True) * cells * 2 * len(its)
        if k == "smooth_coarse" and precision == "mixed":
            lv, cc = [], n // 2
            while cc * cc * cc * 24 * 8 // 7 > 144000 and cc > 1:
                lv.append(cc ** 3)
                cc //= 2
            b = 28.0 * 2 * mgc * sum(lv) * sum(its)
        if b > 0 and kms > 0:
            e["alg_GBs"] = round(b / (kms * 1e-3) / 1e9, 1)
            e["frac"] = round(b / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        out[k] = e
    return out


def copy_bandwidth():
    """HBM rate of torch's device copy (1 GiB read + 1 GiB written per copy,
    10 copies timed with events on torch's stream): context for the roofline
    fraction, which is taken against the published peak."""
    import torch
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / 10
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (1 << 27) * 8 / sec / 1e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_solver(case, precision, steps, warmup, prof_class=None, profile_all=False,
                graph=False, tune=False, knobs=None):
    """Time `steps` steps of one case (or a list of cases: a batch) after
    `warmup` untimed ones; optionally profile every kernel class over one
    extra untimed step, and time one class with HIP events over the timed
    region."""
    import torch
    from paper_2003_08374_amd import dbs

    batch = isinstance(case, (list, tuple))
    log(f"{'batch of %d' % len(case) if batch else case.name}: {precision}"
        f"{' graph' if graph else ''}{' tuned' if tune else ''}")
    s = dbs.BatchSolver(case, precision=precision) if batch else dbs.Solver(case,
                                                                              precision=precision)
    tuning = None
    if knobs:
        s.set_tuning(**knobs)
    if tune:
        s.step(1)
        tuning = s.autotune()
    if graph:
        s.set_graph(True)
        # graph replays settle their iteration budgets over the first steps
        # (one eager step, the capture, four replays with slack, the capture
        # with the shrunk budgets and its first replay): time the steady state
        warmup = max(warmup, 8)
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
        # the most expensive class that has an algorithmic byte model
        modelled = {k: v for k, v in all_times.items() if alg_bytes_per_cell(k, 4) > 0}
        dom = max(modelled.items(), key=lambda kv: kv[1][1])[0] if modelled else None
    if dom and not graph:
        s.set_profiling(1 << dbs.Solver.kernel_class(dom))
    s.reset_profiling()
    stats = (lambda: s.stats(0)) if batch else s.stats
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # one call for all timed steps, as a time loop makes it (the library
    # synchronises and gathers its statistics once per call)
    s.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sts = stats()
    # the last timed step's counts
    its, sweeps = [sts["p_iters"]], [sts["mom_sweeps"]]
    log(f"  {steps} steps in {t1 - t0:.3f} s")
    kt = s.kernel_times()
    st = stats()
    sts_all = [s.stats(i) for i in range(len(case))] if batch else [st]
    if batch:
        its_all = [v["p_iters"] for v in sts_all]
        st["p_iters_max"] = [max(v[c] for v in its_all) for c in range(len(its_all[0]))]
    s.close()
    return {"sec": t1 - t0, "p_iters": its, "sweeps": sweeps, "kernel": dom, "ktimes": kt,
            "all": all_times, "stats": st, "tuning": tuning,
            "invariants": invariants(sts_all, (case[0] if batch else case).p_tol)}


def invariants(sts, p_tol):
    """State checks after the last timed step, over every sample: the
    discrete divergence of the corrected fluxes against the bound the last
    converged pressure solve guarantees (p_tol ||b||), and the range of
    alpha."""
    ratio = max(v["max_div"] / (p_tol * v["p_bnorm"][-1]) if v["p_bnorm"][-1] > 0 else 0.0
                for v in sts)
    amin = min(v["alpha_min"] for v in sts)
    amax = max(v["alpha_max"] for v in sts)
    return {"max_div_over_bound": ratio, "div_within_bound": ratio <= 1.0 + 1e-9,
            "alpha_range": [amin, amax]}


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
        "parity": parity_sample(O, W),
    }


def parity_sample(O, W, n=48, steps=2):
    """Per-field errors of the HIP path against the oracle (untimed, in the
    CPU leg): a 48^3 instance of the benchmark generator, 2 steps, the
    oracle's pressure solves to 1e-14 and the GPU's to 1e-13, FP64 and
    mixed.  Relative L2 on p_rgh, U and F, max-abs on alpha."""
    import numpy as np
    from paper_2003_08374_amd import dbs

    c = W.fractured_3d(n=n, seed_k=3, seed_phi=4, fractures="planes", frac_seed=5, n_frac=3,
                       name=f"fractured_3d_{n}_planes")
    ref, _ = O.step(c.replace(p_tol=1e-14, p_maxit=200000), O.initial_state(c), steps)
    rel = lambda a, b: float(np.linalg.norm(np.ravel(a) - np.ravel(b)) /
                             max(np.linalg.norm(np.ravel(b)), 1e-300))
    out = {"workload": c.name, "steps": steps, "oracle_p_tol": 1e-14, "gpu_p_tol": 1e-13,
           "bar": {"fp64": 1e-10, "mixed": 1e-9}}
    for prec in ("fp64", "mixed"):
        with dbs.Solver(c.replace(p_tol=1e-13), precision=prec) as s:
            s.step(steps)
            g = s.state()
        out[prec] = {
            "alpha_maxabs": float(np.max(np.abs(g["alpha"] - ref["alpha"]))),
            "U_relL2": rel(g["U"], ref["U"]),
            "p_rgh_relL2": rel(g["p_rgh"], ref["p_rgh"]),
            "F_relL2": rel(np.concatenate(g["F"]), np.concatenate(ref["F"])),
        }
    return out


def batch_leg(args):
    """The 512-sample batch (edges U{32..96}, no fracture, k seed 1000+s, phi
    seed 2000+s): mixed precision after autotuning, eagerly and in graph
    mode, and plain FP64 eagerly, all to a relative residual of 1e-8."""
    from paper_2003_08374_amd import workloads as W

    log(f"generating {args.batch_samples} samples")
    cases = W.batch_cases(n_samples=args.batch_samples, seed=6, lo=32, hi=96, p_tol=args.p_tol)
    cases = [c.replace(p_maxit=500, mom_tol=args.mom_tol) for c in cases]
    cells = sum(c.ncells for c in cases)
    out = {"workload": f"batch{len(cases)}_edges32to96", "samples": len(cases), "cells": cells,
           "p_tol": args.p_tol}
    rm = time_solver(cases, "mixed", args.steps, args.warmup, tune=True)
    out["mixed_tuned"] = {"value": cells / (rm["sec"] / args.steps),
                          "ms_per_step": rm["sec"] / args.steps * 1e3,
                          "tuning": rm["tuning"],
                          "p_iters_max_last": rm["stats"].get("p_iters_max"),
                          "invariants": rm["invariants"]}
    rg = time_solver(cases, "mixed", args.steps, args.warmup, graph=True, tune=True)
    out["mixed_graph_tuned"] = {"value": cells / (rg["sec"] / args.steps),
                                "ms_per_step": rg["sec"] / args.steps * 1e3,
                                "tuning": rg["tuning"],
                                "p_iters_max_last": rg["stats"].get("p_iters_max"),
                                "invariants": rg["invariants"]}
    r64 = time_solver(cases, "fp64", args.steps, args.warmup)
    out["fp64_eager"] = {"value": cells / (r64["sec"] / args.steps),
                         "ms_per_step": r64["sec"] / args.steps * 1e3,
                         "p_iters_max_last": r64["stats"].get("p_iters_max"),
                         "invariants": r64["invariants"]}
    out["speedup_mixed_batched_vs_fp64"] = (max(out["mixed_tuned"]["value"],
                                                out["mixed_graph_tuned"]["value"]) /
                                            out["fp64_eager"]["value"])
    return out


def flume_leg(args):
    """The 2D wave flume (2048 x 512, 5 mm cells, dt 1e-3 s) batched over 16
    seeded wave amplitudes, mixed precision after autotuning, eagerly (the
    reported value) and in graph mode, p_tol 1e-8."""
    from paper_2003_08374_amd import workloads as W

    log("generating the flume batch")
    cases = [c.replace(p_maxit=500, mom_tol=args.mom_tol)
             for c in W.flume_batch(n=16, seed=7, p_tol=args.p_tol)]
    cells = sum(c.ncells for c in cases)
    rm = time_solver(cases, "mixed", args.steps, args.warmup, tune=True)
    rg = time_solver(cases, "mixed", args.steps, args.warmup, graph=True, tune=True)
    return {"workload": "wave_flume_2048x512_batch16", "samples": len(cases), "cells": cells,
            "p_tol": args.p_tol, "value": cells / (rm["sec"] / args.steps),
            "ms_per_step": rm["sec"] / args.steps * 1e3, "tuning": rm["tuning"],
            "p_iters_max_last": rm["stats"].get("p_iters_max"),
            "invariants": rm["invariants"],
            "graph_ms_per_step": rg["sec"] / args.steps * 1e3,
            "graph_invariants": rg["invariants"]}


def csf_leg(args, case):
    """The headline 256^3 workload with clear-fluid CSF surface tension on
    (sigma = 0.03 N/m, water-oil), mixed precision, eagerly; the curvature
    kernels are timed with HIP events over the timed steps."""
    cs = case.replace(sigma=0.03)
    r = time_solver(cs, "mixed", args.steps, args.warmup, prof_class="curvature")
    cells = cs.ncells
    launches, kms = r["ktimes"].get("curvature", (0, 0.0))
    ms_k = kms / args.steps
    return {"workload": case.name + "_csf", "sigma": cs.sigma,
            "value": cells / (r["sec"] / args.steps),
            "ms_per_step": r["sec"] / args.steps * 1e3,
            "p_iters_last": r["p_iters"][-1], "invariants": r["invariants"],
            "curvature": {"ms_per_step": round(ms_k, 4), "launches_per_step": launches / args.steps,
                          "alg_bytes_per_cell": alg_bytes_per_cell("curvature", 4),
                          "achieved_GBs": round(alg_bytes_per_cell("curvature", 4) * cells /
                                                (ms_k * 1e-3) / 1e9, 1) if ms_k > 0 else None}}


def reservoir_leg(args):
    """The Darcy-scale heterogeneous reservoir at the paper's 2000 x 800
    cells (block permeabilities 1e-13..4e-13 m^2, water into oil, dt 0.5 s),
    mixed precision, eagerly: a 2D, Darcy-dominated pressure system."""
    from paper_2003_08374_amd import workloads as W

    cs = W.reservoir_2d(nx=2000, ny=800, dt=0.5).replace(p_tol=args.p_tol, p_maxit=500,
                                                          mom_tol=args.mom_tol)
    r = time_solver(cs, "mixed", args.steps, args.warmup)
    return {"workload": cs.name, "cells": cs.ncells, "p_tol": args.p_tol,
            "value": cs.ncells / (r["sec"] / args.steps),
            "ms_per_step": r["sec"] / args.steps * 1e3, "p_iters_last": r["p_iters"][-1],
            "invariants": r["invariants"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=12)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--p-tol", type=float, default=1e-8)
    ap.add_argument("--mom-tol", type=float, default=1e-8,
                    help="momentum predictor tolerance (relative residual)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--kernel", default=None, help="kernel class for the roofline")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-mode leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched leg")
    ap.add_argument("--no-flume", action="store_true", help="skip the wave-flume batch leg")
    ap.add_argument("--no-csf", action="store_true", help="skip the surface-tension leg")
    ap.add_argument("--no-reservoir", action="store_true",
                    help="skip the heterogeneous-reservoir leg")
    ap.add_argument("--batch-samples", type=int, default=512)
    ap.add_argument("--coarse-sweeps", type=int, default=3)
    ap.add_argument("--fused", type=int, default=1,
                    help="1: fused full sweeps on the fine level (else half sweeps)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--summarize-counters", metavar="DIR", default=None,
                    help="print the markdown summary of a rocprofv3 step measurement in DIR "
                         "(trace, fetch, write, cfetch, cwrite) and exit")
    args = ap.parse_args()
    if args.summarize_counters:
        d = args.summarize_counters
        flags = ("--no-cpu --no-fp64 --no-graph --no-batch --no-flume --no-csf --no-reservoir "
                 "--kernel axpy")
        # the default run's warm-up and timed steps
        t = (f"rocprofv3 --kernel-trace --stats --output-format csv -d <out>/trace -o run -- "
             f"python3 <repo>/bench.py {flags} --steps 10 --warmup 12")
        c = "\n".join(f"rocprofv3 --pmc {p} --output-format csv -d <out>/{q} -o run -- python3 "
                      f"<repo>/bench.py {flags} --steps 10 --warmup 12"
                      for p, q in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write"))) + "\n" + \
            "\n".join(f"rocprofv3 --pmc {p} --output-format csv -d <out>/{q} -o run -- python3 "
                      f"<repo>/bench.py --copy-calibration"
                      for p, q in (("FETCH_SIZE", "cfetch"), ("WRITE_SIZE", "cwrite")))
        sys.stdout.write(summarize_counters(d, args.n, args.precision, t, c))
        return

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
    case = case.replace(p_tol=args.p_tol, p_maxit=500, mom_tol=args.mom_tol)
    cells = case.ncells

    knobs = {"kz": 0, "sweeps": 2, "coarse_sweeps": args.coarse_sweeps, "bottom_shift": 0,
             "fused": args.fused}
    main_run = time_solver(case, args.precision, args.steps, args.warmup,
                           prof_class=args.kernel, profile_all=args.kernel is None, knobs=knobs)
    ms = main_run["sec"] / args.steps * 1e3
    value = cells / (main_run["sec"] / args.steps)
    rsize = 4 if args.precision == "mixed" else 8
    kname = main_run["kernel"]
    launches, kms = main_run["ktimes"].get(kname, (0, 0.0))
    per_cell = alg_bytes_per_cell(kname, rsize, bool(args.fused))
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
        # context: the rate of torch's own device copy in the same run
        roof["torch_copy_GBs"] = round(copy_bandwidth(), 1)
    if roof is not None:
        roof["step"] = step_roofline(main_run, cells, args.precision, ms, args.n)
        roof["classes"] = class_table(main_run, cells, args.precision, args.n,
                                      main_run["p_iters"][-1], knobs["coarse_sweeps"])

    fp64 = None
    if not args.no_fp64 and args.precision == "mixed":
        r64 = time_solver(case, "fp64", args.steps, args.warmup, prof_class=kname)
        fp64 = {"value": cells / (r64["sec"] / args.steps),
                "ms_per_step": r64["sec"] / args.steps * 1e3,
                "p_iters_last": r64["p_iters"][-1], "invariants": r64["invariants"]}
    graph = None
    if not args.no_graph:
        rg = time_solver(case, args.precision, args.steps, args.warmup, graph=True)
        graph = {"value": cells / (rg["sec"] / args.steps),
                 "ms_per_step": rg["sec"] / args.steps * 1e3,
                 "p_iters_last": rg["p_iters"][-1], "invariants": rg["invariants"]}
    batched = None if args.no_batch else batch_leg(args)
    flume = None if args.no_flume else flume_leg(args)
    csf = None if args.no_csf else csf_leg(args, case)
    reservoir = None if args.no_reservoir else reservoir_leg(args)
    cpu = None if args.no_cpu else cpu_baseline()

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
        "invariants": main_run["invariants"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64_same_tol": fp64,
        "speedup_mixed_vs_fp64": (value / fp64["value"]) if fp64 else None,
        "graph_mode": graph,
        "batched": batched,
        "flume_batch": flume,
        "csf": csf,
        "reservoir": reservoir,
    }
    if main_run["all"]:
        line["kernel_ms_one_step"] = {k: round(v[1], 3) for k, v in sorted(
            main_run["all"].items(), key=lambda kv: -kv[1][1])}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
