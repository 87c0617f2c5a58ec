"""Continuous-batching serving of independent simulations on one GPU.

A request is a periodic 3-D Euler mesh of 16^3 blocks with a smooth seeded
initial state and a number of CFL steps.  Requests arrive as a Poisson stream;
the batch library (agile_batch_*) admits them first come, first served as pool
memory frees up, advances every resident request by one step per tick in one
batched launch sequence, and hands back finished states.  This module makes
the request stream and drives the ticks; admission, stepping and retirement
happen in the library.

Request recipe (seeded with SplitMix64 through ``workloads.uniform``):
  - block count n* log-uniform in [bmin, bmax]; the mesh is a near-cubic box
    of a x b x c base blocks (max/min side ratio <= 2), either uniform or, for
    a fraction of the requests, with the central (a/2, b/2, c/2) sub-box of
    base blocks refined once (2:1), whichever box gives the leaf count closest
    to n*; cells are cubic, the domain is (a, b, c)/a;
  - steps uniform in [smin, smax];
  - rho = 1.25 + 0.75 S_rho, p = 1.25 + 0.75 S_p, v_d = 0.17 S_vd, where each
    S is a product of three sines sin(2 pi k_d x_d / L_d + phi_d) with k_d in
    {1, 2} and seeded phases: smooth, periodic, rho and p in [0.5, 2], |v| < 0.3.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import workloads as W

BN = 16
CELLS = BN ** 3


@dataclass
class Request:
    tag: int
    blocks: np.ndarray      # int32 [n, 4] (level, ix, iy, iz)
    base: tuple
    hi: tuple
    max_level: int
    steps: int
    seed: int
    gap: float              # exponential(1) inter-arrival gap (scaled by 1/rate)

    @property
    def nblocks(self) -> int:
        return int(self.blocks.shape[0])

    def workload(self, riemann=W.HLLC, gamma=5.0 / 3.0, cfl=0.4) -> W.Workload:
        """The request as a Workload without a host state (U = None)."""
        return W.Workload(f"req{self.tag}", W.EULER, riemann, gamma, cfl, (BN, BN, BN), self.base, (0.0, 0.0, 0.0),
                          self.hi, self.max_level, self.blocks, None, self.steps)


def _box_leaves(a, b, c, refined):
    return a * b * c + (7 * (a // 2) * (b // 2) * (c // 2) if refined else 0)


def _pick_box(target, refined):
    best = None
    for c in range(1, 33):
        for b in range(c, 2 * c + 1):
            for a in range(b, 2 * c + 1):
                if refined and c < 2:
                    continue
                n = _box_leaves(a, b, c, refined)
                d = abs(math.log(n / target))
                if best is None or d < best[0]:
                    best = (d, (a, b, c))
    return best[1]


def _box_blocks(a, b, c, refined):
    blocks = W.uniform_blocks((a, b, c))
    if not refined:
        return blocks
    lo = (a // 4, b // 4, c // 4)
    hi = (lo[0] + a // 2, lo[1] + b // 2, lo[2] + c // 2)
    inside = [q for q, (_, x, y, z) in enumerate(blocks.tolist())
              if lo[0] <= x < hi[0] and lo[1] <= y < hi[1] and lo[2] <= z < hi[2]]
    return W.refine_blocks(blocks, inside)


def make_requests(n=512, seed=11, bmin=8, bmax=4096, smin=20, smax=200, refine_frac=0.5):
    """The seeded request stream (host only: meshes, step counts, seeds, gaps)."""
    q = np.arange(n)
    u_size = W.uniform01(seed, q, 0)
    u_ref = W.uniform01(seed, q, 1)
    u_steps = W.uniform01(seed, q, 2)
    u_gap = W.uniform01(seed, q, 3)
    reqs = []
    for i in range(n):
        target = math.exp(math.log(bmin) + (math.log(bmax) - math.log(bmin)) * u_size[i])
        refined = bool(u_ref[i] < refine_frac) and target >= 15
        a, b, c = _pick_box(target, refined)
        if refined and (a // 2) * (b // 2) * (c // 2) == 0:
            refined = False
        blocks = _box_blocks(a, b, c, refined)
        steps = smin + min(int(u_steps[i] * (smax - smin + 1)), smax - smin)
        reqs.append(Request(i, blocks, (a, b, c), (1.0, b / a, c / a), 2 if refined else 1, steps,
                            seed * 1000003 + i, -math.log1p(-u_gap[i])))
    return reqs


def initial_state(req: Request, device="cuda", gamma=5.0 / 3.0):
    """Conserved initial state [n, 5, 16, 16, 16] (float64 torch tensor) built on `device`."""
    import torch
    blk = torch.as_tensor(req.blocks.astype(np.int64), device=device)
    lev = blk[:, 0]
    dx = (1.0 / (req.base[0] * BN)) / torch.pow(2.0, (lev - 1).to(torch.float64))
    L = (1.0, req.hi[1], req.hi[2])
    r = W.uniform01(req.seed, np.arange(30), 5)
    ii = torch.arange(BN, device=device, dtype=torch.float64) + 0.5

    def sines(f):
        out = []
        for d in range(3):
            k = 1.0 + float(r[6 * f + 2 * d] < 0.5)
            ph = 2.0 * math.pi * float(r[6 * f + 2 * d + 1])
            x = (blk[:, 1 + d].to(torch.float64)[:, None] * BN + ii[None, :]) * dx[:, None]
            out.append(torch.sin((2.0 * math.pi * k / L[d]) * x + ph))
        sx, sy, sz = out
        return sz[:, :, None, None] * sy[:, None, :, None] * sx[:, None, None, :]

    rho = 1.25 + 0.75 * sines(0)
    p = 1.25 + 0.75 * sines(1)
    v = [0.17 * sines(2 + d) for d in range(3)]
    U = torch.empty((req.nblocks, 5, BN, BN, BN), dtype=torch.float64, device=device)
    U[:, 0] = rho
    for d in range(3):
        U[:, 1 + d] = rho * v[d]
    U[:, 4] = p / (gamma - 1.0) + 0.5 * rho * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2])
    return U


def mean_work(reqs) -> float:
    """Mean cell-updates per request (cells x steps)."""
    return float(np.mean([r.nblocks * CELLS * r.steps for r in reqs]))


def percentile_weighted(values, weights, q):
    """q-th percentile of `values` each repeated `weights` times (nearest rank)."""
    v = np.asarray(values, dtype=np.float64)
    w = np.asarray(weights, dtype=np.int64)
    if v.size == 0 or w.sum() == 0:
        return float("nan")
    o = np.argsort(v, kind="stable")
    c = np.cumsum(w[o])
    rank = max(1, int(math.ceil(q / 100.0 * c[-1])))
    return float(v[o][np.searchsorted(c, rank)])


def serve(batch, reqs, rate, stream=None, device="cuda", keep=None, log=None, host_states=False):
    """Run the request stream through `batch` (agile.Batch) with Poisson arrivals
    at `rate` requests/s (wall clock).  Ticks run back to back while requests
    are resident or queued; an idle engine waits for the next arrival.

    stream: the torch stream the batch was created on; initial states are built
    on it, so that the tick that admits a request reads a finished state.
    keep: optional set of tags whose final states are returned (device tensors).
    host_states: build each initial state on the host (float64 ndarray) and
    submit that copy instead of a device tensor (the batch copies it).
    Returns a dict of per-tick and per-request records and summary figures."""
    import torch
    if stream is not None:
        with torch.cuda.stream(stream):
            return _serve(batch, reqs, rate, device, keep, log, host_states)
    return _serve(batch, reqs, rate, device, keep, log, host_states)


def _serve(batch, reqs, rate, device, keep, log, host_states=False):
    import torch
    arrive = np.cumsum([r.gap for r in reqs]) / rate
    by_tag = {r.tag: r for r in reqs}
    out_buf = None
    results = {}
    ticks = []          # (t_start, duration, active requests, active blocks)
    rec = {r.tag: {"arrive": float(arrive[i]), "admit": None, "finish": None} for i, r in enumerate(reqs)}
    waiting = set()     # submitted, not yet finished
    running = set()
    nxt = 0
    t0 = time.perf_counter()
    while nxt < len(reqs) or waiting:
        now = time.perf_counter() - t0
        while nxt < len(reqs) and arrive[nxt] <= now:
            r = reqs[nxt]
            U0 = initial_state(r, "cpu").numpy() if host_states else initial_state(r, device)
            batch.submit(r.workload(batch.riemann), r.steps, r.tag, U=U0)
            waiting.add(r.tag)
            nxt += 1
        if not waiting:
            time.sleep(max(0.0, min(arrive[nxt] - (time.perf_counter() - t0), 0.05)))
            continue
        ts = time.perf_counter()
        info = batch.tick()
        te = time.perf_counter()
        ticks.append((ts - t0, te - ts, info["active"], info["active_blocks"], info["admitted"],
                      info["admit_ms"], info["build_ms"], info["graph_builds"]))
        if info["admitted"] or info["finished"]:
            for tag in list(waiting):
                st, _ = batch.status(tag)
                if st != 1 and rec[tag]["admit"] is None:     # left the queue this tick
                    rec[tag]["admit"] = ts - t0
                    running.add(tag)
                if st == 3:                                      # finished
                    rec[tag]["finish"] = te - t0
                    n = by_tag[tag].nblocks
                    if keep is not None and tag in keep:
                        buf = torch.empty((n, 5, BN, BN, BN), dtype=torch.float64, device=device)
                        _, steps, t = batch.result(tag, out=buf)
                        results[tag] = (buf, steps, t)
                    else:
                        if out_buf is None or out_buf.numel() < n * 5 * CELLS:
                            out_buf = torch.empty(max(n, 4096) * 5 * CELLS, dtype=torch.float64, device=device)
                        batch.result(tag, out=out_buf[:n * 5 * CELLS].view(n, 5, BN, BN, BN))
                    waiting.discard(tag)
                    running.discard(tag)
        if log is not None and len(ticks) % 50 == 0:
            log(f"tick {len(ticks)}: t={te - t0:.2f}s arrived={nxt} waiting={len(waiting)} "
                f"active={info['active']} blocks={info['active_blocks']} queued={info['queued']}")
    t_end = time.perf_counter() - t0
    d = np.array([t[1] for t in ticks])
    act = np.array([t[2] for t in ticks], dtype=np.int64)
    blocks = np.array([t[3] for t in ticks], dtype=np.int64)
    cells = float(blocks.sum()) * CELLS
    lat = np.array([rec[t]["finish"] - rec[t]["arrive"] for t in rec])
    wait = np.array([rec[t]["admit"] - rec[t]["arrive"] for t in rec])
    return {
        "requests": len(reqs),
        "ticks": len(ticks),
        "wall_s": t_end,
        "busy_s": float(d.sum()),
        "cell_updates": cells,
        "aggregate_cell_updates_per_s": cells / (t_end - float(arrive[0])),
        "busy_cell_updates_per_s": cells / float(d.sum()),
        "step_latency_ms": {"p50": 1e3 * percentile_weighted(d, act, 50),
                            "p99": 1e3 * percentile_weighted(d, act, 99),
                            "max": 1e3 * float(d.max())},
        "request_latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "queue_wait_s": {"p50": float(np.percentile(wait, 50)), "p99": float(np.percentile(wait, 99))},
        "mean_active_requests": float(np.average(act, weights=d)) if d.sum() > 0 else 0.0,
        "mean_active_blocks": float(np.average(blocks, weights=d)) if d.sum() > 0 else 0.0,
        # host work inside the ticks: admission (plans, copies of initial
        # states) and step-graph captures after the set of running requests
        # changed
        "graph_builds": int(sum(t[7] for t in ticks)),
        "graph_build_ms_total": float(sum(t[6] for t in ticks)),
        "admit_ms_total": float(sum(t[5] for t in ticks)),
        "results": results,
        "ticks_log": ticks,
    }
