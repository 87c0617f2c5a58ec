"""Regrid of a running request inside a serving batch (agile_batch_regrid), on
an MI355X through the C-ABI: the request regridded in a mix ends bitwise
where the same request ends when it runs and regrids alone on the plain
single-mesh path, its decision equals the oracle's, and its state after the
regrid and the steps that follow is within the FP64 bar of the oracle, which
runs the whole sequence (steps, estimate, decision, transfer, steps) itself.
Twice: with room in the pool (the request stays resident) and without (it
rejoins the queue and is admitted again once the others have left)."""
from __future__ import annotations

import dataclasses
import sys

import numpy as np
import pytest

from oracle import regrid as RG
from oracle.oracle import Oracle
from paper_2607_19277_amd import workloads as W
from parity import TOL_FP64, oracle_cfl_steps, parity_error

pytestmark = pytest.mark.gpu

PRE, POST, VAR, EPS = 2, 2, 4, 0.01


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def agile():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    from paper_2607_19277_amd import agile as A
    A.lib()
    return A


def _mix():
    a = dataclasses.replace(W.sedov(base_blocks=4, nlevels=3), max_level=4)
    b = W.uniform_random(nb=2, riemann=W.HLLC)
    c = W.smooth_random(W.refine_blocks(W.uniform_blocks((2, 2, 2)), [0]), (2, 2, 2), 2, seed=4)
    return a, b, c


def _oracle_sequence(w):
    """The oracle's own run: PRE CFL steps, its estimate, a refine threshold
    in the widest gap of its estimates inside (0.2, 0.8) (so that rounding
    cannot move a block across it), its decision and transfer, POST steps."""
    R1, t1 = oracle_cfl_steps(w, PRE)
    w1 = dataclasses.replace(w, U=R1)
    est = Oracle(w1).lohner(VAR, EPS)
    v = np.sort(np.unique(np.concatenate([est, [0.2, 0.8]])))
    v = v[(v >= 0.2) & (v <= 0.8)]
    g = int(np.argmax(np.diff(v)))
    refine = 0.5 * (v[g] + v[g + 1])
    new, R, P = RG.decide(w.blocks, est, w.base, w.max_level, refine, -1.0)
    U2 = Oracle(w1).remap(new)
    w2 = dataclasses.replace(w, blocks=np.array(new, dtype=np.int32), U=U2)
    R2, t2 = oracle_cfl_steps(w2, POST)
    return refine, new, R2, t1 + t2


def _alone(agile, w, refine):
    m = agile.Mesh.from_workload(w)
    m.step_cfl(PRE)
    m.regrid(refine, -1.0, w.max_level, variable=VAR, eps=EPS)
    m.step_cfl(POST)
    out = m.readback(), m.blocks(), m.time()
    m.close()
    return out


@pytest.mark.parametrize("room", [True, False])
def test_regrid_in_a_mix_equals_alone_and_the_oracle(agile, room):
    a, b, c = _mix()
    refine, new_ref, R_ref, t_ref = _oracle_sequence(a)
    _say(f"room={room}: oracle refines at {refine:.3f}: {a.nblocks} -> {len(new_ref)} blocks")
    assert len(new_ref) > a.nblocks
    per = 456_100                                  # pool bytes per block incl. ghost slab / register share
    budget = (1 << 30) if room else int(per * (len(new_ref) + 8.5))
    B = agile.Batch(riemann=W.HLLC, budget_bytes=budget)
    cap = B.capacity()[0]
    if not room:      # the grown request fits alone, not beside the other two
        assert len(new_ref) <= cap < len(new_ref) + b.nblocks + c.nblocks, cap
    steps = {0: PRE + POST, 1: 5, 2: 6}
    for tag, w in enumerate((a, b, c)):
        B.submit(w, steps[tag], tag)
    for _ in range(PRE):
        B.tick()
    assert B.status(0) == (agile.REQ_RUNNING, PRE)
    st = B.regrid(0, refine, -1.0, a.max_level, variable=VAR, eps=EPS)
    assert st["new_blocks"] == len(new_ref) and st["refined"] > 0
    assert [tuple(r) for r in B.blocks(0).tolist()] == new_ref
    state, done = B.status(0)
    _say(f"  after the regrid: state {state}, {done} steps taken, capacity {cap}")
    assert done == PRE and state == (agile.REQ_RUNNING if room else agile.REQ_QUEUED)
    res = {}
    for _ in range(40):
        B.tick()
        for tag in range(3):
            if tag not in res and B.status(tag)[0] == agile.REQ_FINISHED:
                res[tag] = B.result(tag)
        if len(res) == 3:
            break
    assert len(res) == 3
    B.close()
    U, n, t = res[0]
    assert n == PRE + POST
    U_alone, blocks_alone, t_alone = _alone(agile, a, refine)
    assert [tuple(r) for r in blocks_alone.tolist()] == new_ref
    assert np.array_equal(U, U_alone) and t == t_alone
    err = parity_error(U, R_ref, a.gamma).max()
    _say(f"  request 0: bitwise equal alone, oracle err {err:.2e}")
    assert err <= TOL_FP64
    assert abs(t - t_ref) <= 1e-12 * t_ref
    for tag, w in ((1, b), (2, c)):
        m = agile.Mesh.from_workload(w)
        m.step_cfl(steps[tag])
        assert np.array_equal(res[tag][0], m.readback()), tag
        m.close()
