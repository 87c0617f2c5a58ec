"""Continuous batching on an MI355X, through the C-ABI: a Poisson stream of
independent requests of uneven size (uniform and 2:1-refined meshes) arrives
while others run; every result must be bitwise the state the same request
reaches when it runs alone on the plain single-mesh path, and within the
FP64 bar of the CPU oracle run for the same number of CFL steps (the
FP32-flux form within 1e-5 in relative L1 of density and energy)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from parity import TOL_FP64, l1_rel, oracle_cfl_steps, parity_error

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision,graph", [(0, True), (1, False)])
def test_stream_results_equal_alone(precision, graph):
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    from paper_2607_19277_amd import agile, serving as S
    reqs = S.make_requests(n=12, seed=5, bmin=8, bmax=96, smin=3, smax=9)
    assert any(r.max_level == 2 for r in reqs) and any(r.max_level == 1 for r in reqs)
    s = torch.cuda.Stream()
    # a pool too small for the whole stream at once: requests queue, then join
    b = agile.Batch(riemann=agile.HLLC, precision=precision, budget_bytes=200 * 460_000, use_graph=graph,
                    autotune=graph, stream=s)
    _say(f"stream of {len(reqs)} requests, pool {b.capacity()[0]} blocks, "
         f"sizes {[r.nblocks for r in reqs]}")
    res = S.serve(b, reqs, rate=400.0, stream=s, keep={r.tag for r in reqs}, host_states=True)
    assert res["requests"] == len(reqs) and len(res["results"]) == len(reqs)
    assert res["mean_active_requests"] > 1.0          # work of several requests overlapped
    b.close()
    for r in reqs:
        Ub, steps, t = res["results"][r.tag]
        assert steps == r.steps
        m = agile.Mesh(agile.EULER, agile.HLLC, precision, 5.0 / 3.0, 0.4, 0.5, r.base, (0, 0, 0), r.hi,
                       r.max_level, stream=s)
        U0 = S.initial_state(r, "cpu").numpy()
        m.set_blocks(r.blocks, U0)
        m.step_cfl(r.steps)
        ref = m.readback()
        assert m.time() == t, r.tag
        torch.cuda.synchronize()
        Uh = Ub.cpu().numpy()
        assert np.array_equal(Uh, ref), r.tag
        m.close()
        w = r.workload()
        w.U = U0
        R, t_ref = oracle_cfl_steps(w, r.steps)
        assert abs(t - t_ref) <= (1e-12 if precision == 0 else 1e-6) * t_ref, (r.tag, t, t_ref)
        if precision == 0:
            err = parity_error(Uh, R, w.gamma).max()
            assert err <= TOL_FP64, (r.tag, err)
        else:
            err = max(l1_rel(Uh[:, 0], R[:, 0]), l1_rel(Uh[:, 4], R[:, 4]))
            assert err <= 1e-5, (r.tag, err)
        _say(f"request {r.tag}: {r.nblocks} blocks (level {r.max_level}), {steps} steps, bitwise equal alone, "
             f"oracle err {err:.2e}")
    _say(f"step latency p50 {res['step_latency_ms']['p50']:.3f} ms, p99 {res['step_latency_ms']['p99']:.3f} ms")
