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
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
# algorithmic bytes per cell of each stage: the first reads U^n and writes
# U^(1); every later one reads its input and U^n and writes its output
# (five FP64 variables for Euler, nine for MHD)
def alg_bytes_stages(nvar, rk):
    return [2 * nvar * 8] + [3 * nvar * 8] * (rk - 1)


# the paper's single-device figures (Table 4: uniform 3-D hydrodynamics, LF,
# van Leer, three-step RK, FP64) in updates per RK substep per second, by block
# edge and domain edge; None: out of memory in the paper
_DEV = ("B200", "GH200", "H100 SXM5 96GB", "A100 SXM4 80GB", "MI250X (1 GCD)")
PAPER_TABLE4 = {
    16: {128: (12.2e8, 8.4e8, 7.94e8, 5.06e8, 1.66e8),
         256: (15.52e8, 11.14e8, 10.32e8, 6.45e8, 1.88e8),
         512: (16.30e8, 10.70e8, 10.86e8, 6.70e8, None)},
    32: {128: (3.04e8, 3.13e8, 3.10e8, 2.58e8, 1.54e8),
         256: (16.24e8, 10.72e8, 10.05e8, 6.67e8, 2.16e8),
         512: (19.91e8, 13.98e8, 13.01e8, 8.28e8, 2.16e8)},
    64: {128: (0.43e8, 0.44e8, 0.44e8, 0.37e8, 0.35e8),
         256: (3.37e8, 3.46e8, 3.39e8, 2.86e8, 1.80e8),
         512: (18.10e8, 11.65e8, 11.08e8, 7.39e8, 2.23e8)},
}


def workload(name, n=256, bn=16):
    from paper_2607_19277_amd import workloads as W
    if name in ("kh", "paper", "srhd") and n not in (128, 256, 512):
        raise SystemExit("--n: 128, 256 or 512")
    if bn not in (16, 32, 64) or (bn != 16 and name not in ("kh", "paper")):
        raise SystemExit("--block: 16, 32 or 64 (32 and 64 with --config kh or paper)")
    if name == "sedov":
        return W.sedov(base_blocks=8, nlevels=4, riemann=W.HLLC), "sedov128_L4_hllc"
    sfx = "" if bn == 16 else f"_b{bn}"
    if name == "kh":
        return W.kelvin_helmholtz(n=n, bn=bn), f"kh{n}_hllc{sfx}"
    if name == "uniform":
        return W.uniform_random(nb=4, riemann=W.HLL), "uniform64_hll"
    if name == "ot":
        # refined on the density of the evolved vortex: the base grid only
        # here, the levels are made on the device (ot_density_mesh)
        return W.orszag_tang(blocks=W.uniform_blocks((8, 8, 2))), "ot128_L4_rho_mhd_hll"
    if name == "ot_jz":
        # the static mesh refined on the initial current density at t = 0
        return W.orszag_tang(), "ot128_L4_mhd_hll"
    if name == "paper":
        # the benchmark numerics of Sec. 3.1 on the double shear layer
        w = W.kelvin_helmholtz(n=n, bn=bn)
        w.riemann, w.limiter, w.rk = W.LF, W.VANLEER, 3
        return w, f"kh{n}_lf_vanleer_rk3{sfx}"
    if name == "srhd":
        # relativistic shear layer with the same numerics (Sec. 3.1; SRHD takes LF, Table 1)
        w = W.srhd_kelvin_helmholtz(n=n)
        w.limiter, w.rk = W.VANLEER, 3
        return w, f"srhd_kh{n}_lf_vanleer_rk3"
    raise SystemExit(f"unknown config {name}")


# Orszag-Tang mesh refined on the density: fraction of the finest level's
# blocks refined in each of the three regrid rounds (with 2:1 balance about
# 21 k leaves, 88 M cells, on a 128 x 128 x 32 base)
OT_RHO_FRACTIONS = (0.8, 0.7, 0.45)


def ot_density_mesh(agile, w, stream, t_end=0.5, fractions=OT_RHO_FRACTIONS, log=None):
    """The vortex on its base grid (w: one level) advanced on the device to
    t_end, then one regrid round per entry of `fractions`: the Loehner
    estimate of the density (the paper's estimator) of every block, and the
    blocks of the finest level whose estimate lies in the top `fraction`
    (and any coarser block above the same value) refined, 2:1 balance
    enforced, the state carried to the new leaves.  Returns the mesh, held
    fixed afterwards."""
    m = agile.Mesh.from_workload(w, stream=stream)
    n = 0
    while m.time() < t_end:
        m.step_cfl(1)
        n += 1
    for r, f in enumerate(fractions):
        est = m.error(0)
        lev = m.blocks()[:, 0]
        fine = est[lev == lev.max()]
        thr = float(np.quantile(fine, 1.0 - f))
        st = m.regrid(thr, -1.0, min(r + 2, w.max_level), variable=0)
        if log:
            log(f"# density regrid {r + 1}: threshold {thr:.4g}, {st['old_blocks']} -> {st['new_blocks']} blocks")
    if log:
        log(f"# {n} base-grid steps to t = {m.time():.4f}")
    return m


def kernel_source_hash(physics="euler"):
    """Hash of the sources of the stage kernel a workload runs (k_stage for
    Euler and SRHD, k_mhd_stage for MHD) with comments and blank space
    removed (the sources hold no string literals), so that a comment edit
    does not mark the stored counter figures stale."""
    h = hashlib.sha256()
    main = "mhd.hip" if physics == "mhd-glm" else "stage.hip"
    for f in (main, "device_math.hpp", "agile_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2607_19277_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update("\n".join(" ".join(l.split()) for l in src.splitlines() if l.strip()).encode())
    return h.hexdigest()[:16]


def stored_traffic(wname, precision, physics="euler"):
    """HBM bytes per stage launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "stage_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(f"{wname}:{precision}")
        if e and e.get("kernel_hash") == kernel_source_hash(physics):
            return e["bytes_per_launch"]
    except Exception:
        return None
    return None


def replace_workload(w, **kw):
    import dataclasses
    return dataclasses.replace(w, **kw)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(w, threads, budget_s, max_steps):
    """Cell-updates/s of the oracle on `threads` host threads: as many full
    steps as fit in the budget (at least one)."""
    from oracle import oracle as orc
    orc.set_threads(threads)
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
    return w.ncells * steps / el, steps, el, orc.threads()


def cpu_baseline(w, budget_s=20.0, max_steps=40, budget_1t_s=10.0):
    """The CPU oracle (plain FP64 C, OpenMP) on the same workload: on every
    host thread this process may use, then on one thread (at least one full
    step each)."""
    v, steps, el, cores = _oracle_rate(w, len(os.sched_getaffinity(0)), budget_s, max_steps)
    v1, steps1, el1, _ = _oracle_rate(w, 1, budget_1t_s, max_steps)
    return {"value": v, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} full SSP-RK{w.rk} steps (dt reduction included) of {w.name} ({w.nblocks} blocks, "
                      f"{w.ncells} cells), {el:.1f} s",
            "value_1thread": v1, "sample_1thread": f"{steps1} full steps on 1 thread, {el1:.1f} s",
            "cpu_model": cpu_model()}


def copy_bandwidth(stream, nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth: the library's streaming copy of nbytes,
    timed with HIP events on `stream` (read + write bytes per second)."""
    import torch
    from paper_2607_19277_amd import agile
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        agile.copy_probe(b, a, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        agile.copy_probe(b, a, stream)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9, ms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="sedov",
                    choices=["sedov", "kh", "uniform", "ot", "ot_jz", "paper", "srhd", "serving", "sedov_amr"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32flux"])
    ap.add_argument("--n", type=int, default=256, help="kh / paper / srhd: domain edge in cells (128, 256, 512)")
    ap.add_argument("--block", type=int, default=16, help="kh / paper: cells per block edge (16, 32, 64)")
    ap.add_argument("--regrid-every", type=int, default=10, help="sedov_amr: steps between regrids")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true", help="also run a plain copy of known size (counter scale)")
    ap.add_argument("--load", type=float, default=0.7, help="serving: offered load / measured service rate")
    ap.add_argument("--requests", type=int, default=512, help="serving: number of requests")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serving: device pool budget (GiB)")
    ap.add_argument("--max-active-blocks", type=int, default=4096,
                    help="serving: step-latency budget of admission in blocks (0: memory only)")
    ap.add_argument("--no-graph", action="store_true", help="serving: eager launches instead of graph replay")
    ap.add_argument("--no-autotune", action="store_true", help="serving: fixed stage shape (no tuner run)")
    ap.add_argument("--autotune", action="store_true", help="single mesh: stage shapes from the tuner")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.config == "serving":
        return serving_main(args)
    if args.config == "sedov_amr":
        return amr_main(args)

    w, wname = workload(args.config, args.n, args.block)      # arguments are checked before any GPU work
    import torch
    from paper_2607_19277_amd import agile

    torch.cuda.set_device(0)
    prec = agile.FP64 if args.precision == "fp64" else agile.FP32_FLUX
    stream = torch.cuda.current_stream()
    print(f"# workload {wname}: {w.nblocks} blocks, {w.ncells} cells, precision {args.precision}", file=sys.stderr,
          flush=True)
    if args.config == "ot":
        say = lambda msg: print(msg, file=sys.stderr, flush=True)
        m0 = ot_density_mesh(agile, w, stream, log=say)
        blocks, U = m0.blocks(), m0.readback()
        t_start = m0.time()
        m0.close()
        w = replace_workload(w, blocks=blocks, U=U)
        say(f"# mesh refined on the density at t = {t_start:.4f}: {w.nblocks} blocks, {w.ncells} cells, levels "
            f"{sorted(set(w.blocks[:, 0].tolist()))}")
    m = agile.Mesh.from_workload(w, precision=prec, stream=stream)
    # stage shapes: the library's default (the plain workgroup order, slab
    # depth from the block count: within 1% of the fastest whole-step shape
    # on every workload measured), or with --autotune the library's tuner
    # (every shape gives bitwise the same cells; where shapes lie within 1%
    # its choice can differ from run to run, and the profiled passes of a
    # workload should run identical launches)
    shapes = m.tune() if args.autotune and w.physics != 1 else None   # the MHD stage has one shape
    for _ in range(args.warmup):
        m.step_cfl(1)
    torch.cuda.synchronize()

    if args.copy_probe:
        # a plain streaming copy of 512 MiB (the counter scale of a profile)
        a = torch.ones(64 * 2 ** 20, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        agile.copy_probe(b, a, stream)
        torch.cuda.synchronize()
        del a, b
    copy_gbs, copy_ms = copy_bandwidth(stream)

    K = args.steps
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    # timed region: HIP events around each step, and around the stage
    # launches of every SAMPLE-th step (a step with kernel events launches
    # eagerly and waits for each event: timing every step's stages costs 3%
    # of the step rate on Sedov, one step in five 0.7%); the other steps
    # replay the step graph captured during the warm-up
    SAMPLE = 5
    m.profile(True, kinds=[agile.K_STAGE])
    m.profile(False, keep=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(K):
        if s % SAMPLE == 0:
            m.profile(True, kinds=[agile.K_STAGE], keep=True)
        starts[s].record(stream)
        m.step_cfl(1)
        ends[s].record(stream)
        if s % SAMPLE == 0:
            m.profile(False, keep=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms, stage_n = m.profile_read(agile.K_STAGE)
    stage_steps = (K + SAMPLE - 1) // SAMPLE
    # breakdown of the other kernel classes: a second, separately timed run
    KB = min(K, 20)
    m.profile(True)
    for s in range(KB):
        m.step_cfl(1)
    fill_ms, _ = m.profile_read(agile.K_FILL)
    reflux_ms, _ = m.profile_read(agile.K_REFLUX)
    dt_ms, _ = m.profile_read(agile.K_DT)
    m.profile(False)
    fill_ms, reflux_ms, dt_ms = fill_ms * K / KB, reflux_ms * K / KB, dt_ms * K / KB
    lat = np.array([starts[s].elapsed_time(ends[s]) for s in range(K)])
    dt_last = m.last_dt()
    print(f"# last dt {dt_last:.4e}; kernel ms/step: stage {stage_ms / stage_steps:.3f} fill {fill_ms / K:.3f} "
          f"reflux {reflux_ms / K:.3f} dt {dt_ms / K:.3f}; step p50 {np.percentile(lat, 50):.3f} ms",
          file=sys.stderr, flush=True)

    value = w.ncells * K / wall
    ms_per_step = wall * 1e3 / K
    avg_stage_s = stage_ms / stage_n / 1e3
    ab = alg_bytes_stages(w.nvar, w.rk)
    alg_bytes = w.ncells * sum(ab) / len(ab)
    achieved = alg_bytes / avg_stage_s / 1e9
    traffic = stored_traffic(wname, args.precision, ["euler", "mhd-glm", "srhd"][w.physics])
    step_alg = w.ncells * sum(ab)          # algorithmic bytes of one whole step
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
        "config": {"workload": wname, "blocks": w.nblocks, "cells": w.ncells, "block": f"{w.bn[0]}^3+2 ghosts",
                   "levels": int(w.blocks[:, 0].max()), "riemann": ["HLL", "HLLC", "LF"][w.riemann],
                   "limiter": ["minmod", "van Leer"][w.limiter], "rk_stages": w.rk,
                   "physics": ["euler", "mhd-glm", "srhd"][w.physics],
                   "precision": args.precision, "dt": "CFL 0.4 on device",
                   "stage_shapes": None if shapes is None else
                   {"kslab": shapes[0], "xcd": shapes[1], "kslab_last": shapes[2], "xcd_last": shapes[3]}},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
        "paper_style_updates_per_s": w.rk * value,
        "kernel_ms_per_step": {"stage": stage_ms / stage_steps, "fill": fill_ms / K, "reflux": reflux_ms / K, "dt": dt_ms / K},
        "roofline": {"bound": "hbm", "kernel": "k_mhd_stage" if w.physics == 1 else "k_stage",
                     "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": avg_stage_s * 1e3,
                     # (i) counter bytes of a stage launch (stored profile of this kernel source) over its time
                     "frac_traffic": (traffic / avg_stage_s / 1e9 / PEAK_HBM_GBS) if traffic else None,
                     # (ii) algorithmic bytes of the whole step (all kernels) at the measured step rate
                     "frac_alg_step": step_alg * K / wall / 1e9 / PEAK_HBM_GBS,
                     "alg_bytes_per_cell_step": sum(ab),
                     "achievable_copy_GBs": copy_gbs, "copy_probe_ms_per_GiB": copy_ms},
    }
    if args.config == "paper":
        ctx = {"unit": "cell-updates per RK substep per s", "ours": w.rk * value}
        ctx[f"paper_table4_{args.n}^3_{args.block}^3_fp64"] = dict(zip(_DEV, PAPER_TABLE4[args.block][args.n]))
        out["paper_context"] = ctx
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle on the host cores ...", file=sys.stderr, flush=True)
        if w.physics == 1:
            # the oracle needs about a minute per step of the full mesh: time
            # the same physics on the 64^2 x 16 base grid with the current-
            # density refinement to three levels (576 leaves, 2.4 M cells)
            from paper_2607_19277_amd import workloads as W
            out["cpu_baseline"] = cpu_baseline(W.orszag_tang(base=(4, 4, 1), nlevels=3, threshold=0.45, step=0.0),
                                               max_steps=10)
        else:
            out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


def amr_main(args):
    """The Sedov mesh with dynamic AMR: a regrid (density estimate, refine /
    coarsen, transfer, table rebuild) every --regrid-every steps inside the
    timed region; value = leaf-cell updates per second including the regrids."""
    import torch
    from paper_2607_19277_amd import agile, workloads as W
    torch.cuda.set_device(0)
    w = W.sedov(base_blocks=8, nlevels=4, riemann=W.HLLC)
    prec = agile.FP64 if args.precision == "fp64" else agile.FP32_FLUX
    stream = torch.cuda.current_stream()
    refine, coarsen, every = 0.05, 0.005, args.regrid_every
    m = agile.Mesh.from_workload(w, precision=prec, stream=stream)
    for _ in range(args.warmup):
        m.step_cfl(1)
    m.regrid(refine, coarsen, w.max_level)
    m.step_cfl(1)
    torch.cuda.synchronize()
    K = args.steps
    ab = alg_bytes_stages(w.nvar, w.rk)
    cells = 0
    stage_ms = stage_bytes = 0.0
    regrid_ms = []
    blocks_seen = [m.n]

    def close_segment():
        nonlocal stage_ms, stage_bytes
        ms, n = m.profile_read(agile.K_STAGE)
        stage_ms += ms
        stage_bytes += m.n * 4096 * sum(ab) / len(ab) * n

    m.profile(True, kinds=[agile.K_STAGE])
    t0 = time.perf_counter()
    for s in range(K):
        m.step_cfl(1)
        cells += m.n * 4096
        if (s + 1) % every == 0 and s + 1 < K:
            close_segment()
            r0 = time.perf_counter()
            m.regrid(refine, coarsen, w.max_level)
            torch.cuda.synchronize()
            regrid_ms.append((time.perf_counter() - r0) * 1e3)
            blocks_seen.append(m.n)
            m.profile(True, kinds=[agile.K_STAGE])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    close_segment()
    m.profile(False)
    achieved = stage_bytes / (stage_ms / 1e3) / 1e9
    out = {
        "metric": "cell-updates/s (Mzone-cycles/s) + % HBM roofline; p50/p99 step latency",
        "value": cells / wall, "unit": "cell-updates/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 flux / f64 state", "data": "synthetic",
        "config": {"workload": "sedov128_L4_hllc_dynamic_amr", "regrid": f"every {every} steps, density "
                   f"estimate, refine > {refine}, coarsen < {coarsen}", "levels": w.max_level,
                   "blocks": blocks_seen, "precision": args.precision},
        "regrid_ms": {"mean": float(np.mean(regrid_ms)) if regrid_ms else None,
                      "max": float(np.max(regrid_ms)) if regrid_ms else None, "count": len(regrid_ms)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "k_stage (all mesh segments)"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


def serving_main(args):
    """Continuous-batching serving of a Poisson stream of independent requests
    (log-uniform 8..4096 blocks, 20..200 steps each); one JSON line."""
    import torch
    from paper_2607_19277_amd import agile, serving as S

    torch.cuda.set_device(0)
    prec = agile.FP64 if args.precision == "fp64" else agile.FP32_FLUX
    reqs = S.make_requests(n=args.requests)
    work = S.mean_work(reqs)
    stream = torch.cuda.Stream()
    mk = lambda cap=args.max_active_blocks: agile.Batch(
        riemann=agile.HLLC, precision=prec, budget_bytes=int(args.budget_gb * 2 ** 30), max_meshes=args.requests,
        use_graph=not args.no_graph, autotune=not args.no_autotune, stream=stream, max_active_blocks=cap)
    # service rate: a saturated batch of the largest requests of another seed
    cal = sorted(S.make_requests(n=64, seed=99), key=lambda r: -r.nblocks)
    b = mk(0)
    tot = 0
    with torch.cuda.stream(stream):
        for r in cal:
            if tot >= 32768:
                break
            b.submit(r.workload(), 1000, r.tag, U=S.initial_state(r))
            tot += r.nblocks
    b.tick()
    b.tick()
    t0 = time.perf_counter()
    cells = 0
    for _ in range(4):
        cells += b.tick()["active_blocks"] * S.CELLS
    mu = cells / (time.perf_counter() - t0)
    b.close()
    rate = args.load * mu / work
    print(f"# serving: {len(reqs)} requests, mean {work / S.CELLS:.0f} block-steps each; service rate "
          f"{mu:.3e} cell-updates/s at {tot} blocks; offered load {args.load} -> {rate:.2f} requests/s",
          file=sys.stderr, flush=True)
    b = mk()
    res = S.serve(b, reqs, rate, stream=stream, log=lambda m: print("# " + m, file=sys.stderr, flush=True))
    cap = b.capacity()[0]
    b.close()
    out = {
        "metric": "cell-updates/s (serving aggregate) + p50/p99 step latency",
        "value": res["aggregate_cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": res["ticks"],
        "warmup": 0,
        "ms_per_step": 1e3 * res["busy_s"] / max(res["ticks"], 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == agile.FP64 else "f32-flux/f64-state",
        "data": "synthetic",
        "config": {"workload": f"serving{len(reqs)}_poisson_load{args.load}", "requests": len(reqs),
                   "blocks_per_request": "log-uniform 8..4096 (uniform or one central 2:1 refined box)",
                   "steps_per_request": "uniform 20..200", "riemann": "HLLC", "precision": args.precision,
                   "pool_blocks": cap, "graph": not args.no_graph, "autotune": not args.no_autotune,
                   "max_active_blocks": args.max_active_blocks,
                   "arrival_rate_per_s": rate, "service_rate_cell_updates_per_s": mu},
        "latency_ms": res["step_latency_ms"],
        "request_latency_s": res["request_latency_s"],
        "queue_wait_s": res["queue_wait_s"],
        "busy_cell_updates_per_s": res["busy_cell_updates_per_s"],
        "wall_s": res["wall_s"],
        "mean_active_requests": res["mean_active_requests"],
        "mean_active_blocks": res["mean_active_blocks"],
        "graph_builds": res["graph_builds"], "graph_build_ms_total": res["graph_build_ms_total"],
        "admit_ms_total": res["admit_ms_total"],
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
