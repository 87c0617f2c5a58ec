"""L1 density / energy error of the HIP path against the FP64 oracle on the
Kelvin-Helmholtz shear layer run to t = 0.5 (the mixed-precision report).

Both sides take the CFL dt of their own state (the same formula) and clip the
last step to land on t_end; the error is sum |U - U_ref| / sum |U_ref| over
all cells, for the density and the total energy.

Full-size use (the oracle's reference takes hours of host time, so it is
written once and compared on the GPU later):
  python tests/kh_l1.py reference --n 256 --block-stride 64 \
      --out tests/golden/kh256_t05_oracle_stride64.npz      (CPU, oracle only)
  python tests/kh_l1.py compare --n 256 --block-stride 64 \
      --ref tests/golden/kh256_t05_oracle_stride64.npz      (GPU, both precisions)
(--physics srhd: the relativistic shear layer, D and tau in place of rho and
e; --block-stride k keeps every k-th block of the (x fastest) block order, so
k = 64 keeps the x = 0 column of blocks at every fourth y and every z: it
crosses both shear layers.)  The reference holds the oracle's density and
energy in float64, so the FP64 path's error is resolved to round-off.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

T_END = 0.5


def oracle_run(w, t_end=T_END, log=None):
    from oracle.oracle import Oracle
    o = Oracle(w)
    t, n = 0.0, 0
    t0 = time.perf_counter()
    while t_end - t > 1e-12:
        dt = min(o.dt(), t_end - t)
        o.step(dt)
        t += dt
        n += 1
        if log and n % 50 == 0:
            log(f"oracle step {n}: t={t:.6f} ({time.perf_counter() - t0:.0f} s)")
    return o.state(), t, n


def gpu_run(w, precision, t_end=T_END):
    from paper_2607_19277_amd import agile
    m = agile.Mesh.from_workload(w, precision=precision)
    t, n = 0.0, 0
    while t_end - t > 1e-12:
        dt = min(m.dt(), t_end - t)
        m.step(dt)
        t += dt
        n += 1
    U = m.readback()
    m.close()
    return U, t, n


def l1_rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["reference", "compare"])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--out")
    ap.add_argument("--ref")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--physics", choices=["euler", "srhd"], default="euler",
                    help="srhd: the relativistic shear layer with LF, van Leer, SSP-RK3")
    ap.add_argument("--block-stride", type=int, default=1,
                    help="store / compare every k-th block only (a smaller reference file)")
    a = ap.parse_args()
    from paper_2607_19277_amd import workloads as W
    if a.physics == "srhd":
        w = W.srhd_kelvin_helmholtz(n=a.n)
        w.limiter, w.rk = W.VANLEER, 3
    else:
        w = W.kelvin_helmholtz(n=a.n)
    sel = slice(None, None, a.block_stride)
    say = lambda s: print(s, flush=True)
    if a.mode == "reference":
        from oracle import oracle as orc
        if a.threads:
            orc.set_threads(a.threads)
        U, t, n = oracle_run(w, log=say)
        np.savez(a.out, rho=U[sel, 0].astype(np.float64), e=U[sel, 4].astype(np.float64), t=t, steps=n,
                 n=a.n, block_stride=a.block_stride, physics=a.physics)
        say(f"reference written: {n} steps to t={t}")
        return
    import torch
    torch.cuda.set_device(0)
    R = np.load(a.ref)
    for prec, name in ((0, "fp64"), (1, "fp32flux")):
        t0 = time.perf_counter()
        U, t, n = gpu_run(w, prec)
        say(f"{w.name} {name}: {n} steps to t={t:.6f} ({time.perf_counter() - t0:.1f} s); "
            f"L1 rel vs oracle (every {a.block_stride}-th block): var 0 {l1_rel(U[sel, 0], R['rho']):.3e}, "
            f"var 4 {l1_rel(U[sel, 4], R['e']):.3e} (oracle: {int(R['steps'])} steps)")


if __name__ == "__main__":
    main()
