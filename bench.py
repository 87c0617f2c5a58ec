#!/usr/bin/env python3
"""Benchmark of the block-AMR finite-volume update on one MI355X.

A step is one full SSP-RK2 step of the whole hot path on the device: ghost
fills (restriction / prolongation at level jumps), two fused stage updates
(primitives, PLM minmod, Riemann flux, divergence, stage combination), two
coarse-fine flux corrections and the CFL signal-speed reduction that sets the
next dt (computed on the device, no host round trip).

Default workload: 3-D Euler Sedov point blast on a 128^3 base grid (8^3
blocks of 16^3) with 3 static nested 2:1 refinement levels, 1856 leaf blocks
(7.6 M cells), HLLC, FP64.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
ALG_BYTES_STAGE = {1: 80, 2: 120}   # per cell: stage 1 reads U^n, writes U^(1); stage 2 reads U^(1), U^n, writes U^{n+1}


def workload(name):
    from paper_2607_19277_amd import workloads as W
    if name == "sedov":
        return W.sedov(base_blocks=8, nlevels=4, riemann=W.HLLC), "sedov128_L4_hllc"
    if name == "kh":
        return W.kelvin_helmholtz(n=256), "kh256_hllc"
    if name == "uniform":
        return W.uniform_random(nb=4, riemann=W.HLL), "uniform64_hll"
    raise SystemExit(f"unknown config {name}")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("stage.hip", "device_math.hpp", "agile_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2607_19277_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(wname, precision):
    """HBM bytes per stage launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "stage_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(f"{wname}:{precision}")
        if e and e.get("kernel_hash") == kernel_source_hash():
            return e["bytes_per_launch"]
    except Exception:
        return None
    return None


def cpu_baseline(w, budget_s=20.0, max_steps=40):
    """The CPU oracle (plain FP64 C, OpenMP) on the same workload: as many full
    steps as fit in the time budget (at least one)."""
    from oracle import oracle as orc
    n_threads = len(os.sched_getaffinity(0))
    orc.set_threads(n_threads)
    o = orc.Oracle(w)
    t0 = time.perf_counter()
    steps = 0
    while True:
        o.step(o.dt())
        steps += 1
        el = time.perf_counter() - t0
        if steps >= max_steps or el * (steps + 1) / steps > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": w.ncells * steps / el, "unit": "cell-updates/s", "cores": orc.threads(), "kind": "oracle",
            "sample": f"{steps} full SSP-RK2 steps (dt reduction included) of the same {w.nblocks}-block mesh, "
                      f"{el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="sedov", choices=["sedov", "kh", "uniform"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32flux"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true", help="also run a plain copy of known size (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_19277_amd import agile

    torch.cuda.set_device(0)
    w, wname = workload(args.config)
    prec = agile.FP64 if args.precision == "fp64" else agile.FP32_FLUX
    stream = torch.cuda.current_stream()
    print(f"# workload {wname}: {w.nblocks} blocks, {w.ncells} cells, precision {args.precision}", file=sys.stderr,
          flush=True)
    m = agile.Mesh.from_workload(w, precision=prec, stream=stream)
    for _ in range(args.warmup):
        m.step_cfl(1)
    torch.cuda.synchronize()

    if args.copy_probe:
        a = torch.empty(64 * 2 ** 20, dtype=torch.float64, device="cuda")   # 512 MiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    K = args.steps
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    m.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(K):
        starts[s].record(stream)
        m.step_cfl(1)
        ends[s].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms, stage_n = m.profile_read(agile.K_STAGE)
    fill_ms, fill_n = m.profile_read(agile.K_FILL)
    reflux_ms, reflux_n = m.profile_read(agile.K_REFLUX)
    dt_ms, dt_n = m.profile_read(agile.K_DT)
    m.profile(False)
    lat = np.array([starts[s].elapsed_time(ends[s]) for s in range(K)])
    dt_last = m.last_dt()
    print(f"# last dt {dt_last:.4e}; kernel ms/step: stage {stage_ms / K:.3f} fill {fill_ms / K:.3f} "
          f"reflux {reflux_ms / K:.3f} dt {dt_ms / K:.3f}; step p50 {np.percentile(lat, 50):.3f} ms",
          file=sys.stderr, flush=True)

    value = w.ncells * K / wall
    ms_per_step = wall * 1e3 / K
    avg_stage_s = stage_ms / stage_n / 1e3
    alg_bytes = w.ncells * 0.5 * (ALG_BYTES_STAGE[1] + ALG_BYTES_STAGE[2])
    achieved = alg_bytes / avg_stage_s / 1e9
    traffic = stored_traffic(wname, args.precision)
    out = {
        "metric": "cell-updates/s (Mzone-cycles/s) + % HBM roofline; p50/p99 step latency",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == agile.FP64 else "f32-flux/f64-state",
        "data": "synthetic",
        "config": {"workload": wname, "blocks": w.nblocks, "cells": w.ncells, "block": "16^3+2 ghosts",
                   "levels": int(w.blocks[:, 0].max()), "riemann": "HLLC" if w.riemann else "HLL",
                   "precision": args.precision, "dt": "CFL 0.4 on device"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
        "paper_style_updates_per_s": 2 * value,
        "kernel_ms_per_step": {"stage": stage_ms / K, "fill": fill_ms / K, "reflux": reflux_ms / K, "dt": dt_ms / K},
        "roofline": {"bound": "hbm", "kernel": "k_stage", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": avg_stage_s * 1e3},
    }
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle on the host cores ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
