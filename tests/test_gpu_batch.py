"""Batched / graph / autotuned forms of the update, through the C-ABI, on an
MI355X.  Every schedule variant must reproduce the plain single-mesh path
bitwise (same per-cell arithmetic), and every batched result is also checked
against the CPU oracle run for the same number of CFL steps."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2607_19277_amd import workloads as W
from parity import TOL_FP64, l1_rel, oracle_cfl_steps, parity_error

pytestmark = pytest.mark.gpu


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


def meshes():
    return {
        "sedov3": W.sedov(base_blocks=4, nlevels=3),
        "uniform": W.uniform_random(nb=2, riemann=W.HLLC),
        "nested2": W.smooth_random(W.nested_blocks((4, 4, 4), 2), (4, 4, 4), 2, seed=21),
        "corner": W.smooth_random(W.refine_blocks(W.uniform_blocks((2, 2, 2)), [0]), (2, 2, 2), 2, seed=4),
    }


def alone(agile, w, steps, precision=0):
    m = agile.Mesh.from_workload(w, precision=precision)
    m.step_cfl(steps)
    return m.readback(), m.time()


@pytest.mark.parametrize("name", ["sedov3", "uniform"])
def test_stage_shapes_are_bitwise_identical(agile, name):
    w = meshes()[name]
    ref, _ = alone(agile, w, 2)
    for ks in (16, 8, 4):
        for x in (0, 1):
            _say(f"{name} kslab={ks} xcd={x}")
            m = agile.Mesh(w.physics, w.riemann, 0, w.gamma, w.cfl, w.glm_alpha, w.base, w.lo, w.hi, w.max_level)
            m.set_option(agile.OPT_KSLAB, ks)
            m.set_option(agile.OPT_XCD, x)
            m.set_option(agile.OPT_KSLAB_LAST, 16 if ks == 4 else 4)   # a different last-stage shape
            m.set_option(agile.OPT_XCD_LAST, 1 - x)
            m.set_blocks(w.blocks, w.U)
            m.step_cfl(2)
            assert np.array_equal(m.readback(), ref), (ks, x)


def test_graph_replays_match_eager(agile):
    import torch
    w = meshes()["sedov3"]
    s = torch.cuda.Stream()
    g = agile.Mesh.from_workload(w, stream=s)
    g.set_option(agile.OPT_GRAPH, 1)
    e = agile.Mesh.from_workload(w)
    for step in range(5):
        g.step_cfl(1)
        e.step_cfl(1)
        # eager work and synchronisations between the replays
        Ug, Ue = g.readback(), e.readback()
        assert np.array_equal(Ug, Ue), step
        assert g.last_dt() == e.last_dt()
        _say(f"graph replay {step} ok")


@pytest.mark.parametrize("pool", [False, True])
def test_tuner_keeps_state_and_results(agile, pool):
    """The tuner times whole steps on a copy of the state (library memory) or
    single launches (a caller-owned pool): either way the state, the time and
    the next dt are unchanged, and later steps equal the untuned mesh's."""
    import torch
    w = meshes()["nested2"]
    buf = None
    if pool:
        need = agile.plan(w.blocks, riemann=w.riemann, gamma=w.gamma, base_blocks=w.base, lo=w.lo, hi=w.hi,
                          max_level=w.max_level)["device_bytes"]
        buf = torch.zeros(need, dtype=torch.uint8, device="cuda")
    m = agile.Mesh.from_workload(w, pool=buf) if pool else agile.Mesh.from_workload(w)
    m.step_cfl(1)
    before, t0, dt0 = m.readback(), m.time(), m.last_dt()
    ks, x, ksl, xl = m.tune()
    _say(f"pool={pool}: tuned kslab={ks} xcd={x}, last stage kslab={ksl} xcd={xl}")
    assert np.array_equal(m.readback(), before)
    assert m.time() == t0 and m.last_dt() == dt0
    m.step_cfl(2)
    ref, t_ref = alone(agile, w, 3)
    assert np.array_equal(m.readback(), ref) and m.time() == t_ref
    m.close()


@pytest.mark.parametrize("precision,graph", [(0, False), (0, True), (1, True)])
def test_batch_results_equal_alone(agile, precision, graph):
    import torch
    ws = meshes()
    steps = {"sedov3": 3, "uniform": 5, "nested2": 2, "corner": 4}
    s = torch.cuda.Stream() if graph else None
    b = agile.Batch(riemann=W.HLLC, precision=precision, budget_bytes=1 << 30, use_graph=graph, autotune=graph,
                    stream=s)
    for tag, (name, w) in enumerate(ws.items()):
        b.submit(w, steps[name], tag)
    done = {}
    for _ in range(20):
        info = b.tick()
        for tag, name in enumerate(ws):
            if tag not in done and b.status(tag)[0] == agile.REQ_FINISHED:
                done[tag] = b.result(tag)
        if len(done) == len(ws):
            break
    assert len(done) == len(ws), info
    for tag, (name, w) in enumerate(ws.items()):
        U, n, t = done[tag]
        ref, tref = alone(agile, w, steps[name], precision)
        assert n == steps[name]
        assert np.array_equal(U, ref), name
        assert t == tref, (name, t, tref)
        R, t_ref = oracle_cfl_steps(w, steps[name])
        assert abs(t - t_ref) <= (1e-12 if precision == 0 else 1e-6) * t_ref, (name, t, t_ref)
        if precision == 0:
            err = parity_error(U, R, w.gamma).max()
            assert err <= TOL_FP64, (name, err)
        else:
            err = max(l1_rel(U[:, 0], R[:, 0]), l1_rel(U[:, 4], R[:, 4]))
            assert err <= 1e-5, (name, err)
        _say(f"batch {name}: {n} steps, t={t:.6e}, bitwise equal alone, oracle err {err:.2e}")


def test_batch_admission_fcfs_by_footprint(agile):
    ws = meshes()
    big, mid, small = ws["sedov3"], ws["nested2"], ws["uniform"]
    # a pool that holds the big mesh, or the mid and the small one, never big + mid
    per = 456_000                 # pool bytes per block incl. ghost slab / flux register share
    b = agile.Batch(riemann=W.HLLC, budget_bytes=per * 180, use_graph=False)
    cap, free = b.capacity()
    assert big.nblocks <= cap < big.nblocks + mid.nblocks
    b.submit(big, 2, 1)
    b.submit(mid, 1, 2)
    b.submit(small, 1, 3)        # fits beside big, but must wait behind mid (first come, first served)
    i1 = b.tick()
    assert (i1["admitted"], i1["queued"], i1["active"]) == (1, 2, 1)
    assert b.status(1)[0] == agile.REQ_RUNNING and b.status(2)[0] == agile.REQ_QUEUED
    assert b.status(3)[0] == agile.REQ_QUEUED
    i2 = b.tick()
    assert i2["finished"] == 1 and b.status(1)[0] == agile.REQ_FINISHED
    i3 = b.tick()                # finished but not collected: still holds its memory
    assert i3["admitted"] == 0 and i3["active"] == 0
    U1, n1, _ = b.result(1)
    assert n1 == 2 and np.array_equal(U1, alone(agile, big, 2)[0])
    i4 = b.tick()
    assert i4["admitted"] == 2 and i4["active"] == 2
    for tag, w in ((2, mid), (3, small)):
        assert b.status(tag)[0] == agile.REQ_FINISHED
        U, n, _ = b.result(tag)
        assert np.array_equal(U, alone(agile, w, 1)[0])
    assert b.capacity()[1] == cap


def test_batch_rejects_and_cancels(agile):
    ws = meshes()
    b = agile.Batch(riemann=W.HLLC, budget_bytes=460_000 * 40)
    with pytest.raises(agile.AgileError) as e:
        b.submit(ws["sedov3"], 1, 1)          # 176 blocks can never fit in ~40
    assert e.value.code == agile.ENOMEM
    b.submit(ws["uniform"], 3, 7)
    with pytest.raises(agile.AgileError):
        b.submit(ws["uniform"], 3, 7)         # duplicate tag
    b.tick()
    assert b.status(7) == (agile.REQ_RUNNING, 1)
    b.cancel(7)
    assert b.status(7)[0] == agile.REQ_UNKNOWN
    b.submit(ws["corner"], 1, 8)
    info = b.tick()
    assert info["admitted"] == 1 and info["finished"] == 1
    U, n, _ = b.result(8)
    assert np.array_equal(U, alone(agile, ws["corner"], 1)[0])


def test_admission_within_the_step_latency_budget(agile):
    """With max_active_blocks, a request that fits in memory still waits while
    the running requests' blocks plus its own exceed the budget; an idle batch
    always admits its head, and results stay bitwise those of the requests
    alone."""
    ws = meshes()
    big, mid, small = ws["sedov3"], ws["nested2"], ws["uniform"]   # 176, 120, 8 blocks
    b = agile.Batch(riemann=W.HLLC, budget_bytes=1 << 30, max_active_blocks=180)
    b.submit(big, 2, 1)
    b.submit(small, 1, 2)      # 176 + 8 > 180: waits although memory is plentiful
    b.submit(mid, 1, 3)
    i1 = b.tick()
    assert (i1["admitted"], i1["active_blocks"]) == (1, big.nblocks)
    assert b.status(2)[0] == agile.REQ_QUEUED and b.status(3)[0] == agile.REQ_QUEUED
    i2 = b.tick()              # big still running at the start of the tick
    assert i2["admitted"] == 0 and i2["finished"] == 1
    i3 = b.tick()              # big finished (inactive, not collected): 8 + 120 <= 180
    assert i3["admitted"] == 2 and i3["active_blocks"] == small.nblocks + mid.nblocks
    for tag, w, n in ((1, big, 2), (2, small, 1), (3, mid, 1)):
        U, steps, _ = b.result(tag)
        assert steps == n and np.array_equal(U, alone(agile, w, n)[0]), tag
    one = agile.Batch(riemann=W.HLLC, budget_bytes=1 << 30, max_active_blocks=16)
    one.submit(big, 1, 9)      # larger than the budget: admitted into the idle batch
    assert one.tick()["admitted"] == 1
    assert np.array_equal(one.result(9)[0], alone(agile, big, 1)[0])
