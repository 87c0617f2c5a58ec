"""Caller-owned device memory (agile_config.dev_pool) on an MI355X, through the
C-ABI: a mesh and a serving batch whose every device array lives in a torch
tensor give bitwise the results of the library-allocated path; a regrid that
outgrows the caller's pool is refused without harm and succeeds in a larger
pool, equal to the library-allocated regrid."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2607_19277_amd import workloads as W

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


def _need(agile, w):
    return agile.plan(w.blocks, physics=w.physics, riemann=w.riemann, base_blocks=w.base, lo=w.lo, hi=w.hi,
                      max_level=w.max_level, rk_stages=getattr(w, "rk", 2))["device_bytes"]


@pytest.mark.parametrize("graph", [False, True])
def test_mesh_in_a_torch_pool_equals_library_allocation(agile, graph):
    import torch
    w = W.sedov(base_blocks=4, nlevels=3)
    s = torch.cuda.Stream()
    need = _need(agile, w)
    pool = torch.zeros(need, dtype=torch.uint8, device="cuda")
    _say(f"sedov3 in a {need} byte pool, graph={graph}")
    m = agile.Mesh.from_workload(w, stream=s, pool=pool)
    r = agile.Mesh.from_workload(w, stream=s)
    for x in (m, r):
        x.set_option(agile.OPT_GRAPH, int(graph))
    for k in range(3):
        m.step_cfl(1)
        r.step_cfl(1)
        U = m.readback()
        assert np.array_equal(U, r.readback()), k
        assert m.last_dt() == r.last_dt()
    # the state lives in the tensor: its first array is U^n in the device order
    torch.cuda.synchronize()
    n = w.nblocks * 5 * 4096
    head = pool[:8 * n].view(torch.float64).cpu().numpy()
    assert np.array_equal(np.sort(head), np.sort(U.ravel()))
    m.close()
    r.close()


def test_regrid_in_a_caller_pool(agile):
    """An exact-size pool leaves no room to refine: the regrid returns
    AGILE_ENOMEM, the mesh keeps its blocks and state and steps on.  In a pool
    four times larger the same regrid succeeds, equal to the regrid of a
    library-allocated mesh, with time and dt carried over."""
    import dataclasses
    import torch
    w = dataclasses.replace(W.smooth_random(W.nested_blocks((4, 4, 4), 2), (4, 4, 4), 2, seed=21), max_level=3)
    need = _need(agile, w)
    small = torch.empty(need, dtype=torch.uint8, device="cuda")
    m = agile.Mesh.from_workload(w, pool=small)
    m.step_cfl(2)
    err = m.error(4)
    refine, coarsen = float(np.quantile(err, 0.8)), float(np.quantile(err, 0.05))
    before = m.readback()
    with pytest.raises(agile.AgileError) as e:
        m.regrid(refine, coarsen, 3, variable=4)
    assert e.value.code == agile.ENOMEM
    assert np.array_equal(m.readback(), before) and np.array_equal(m.blocks(), np.asarray(w.blocks))
    m.step_cfl(1)                                  # not a sticky error
    m.close()
    big = torch.empty(4 * need, dtype=torch.uint8, device="cuda")
    a = agile.Mesh.from_workload(w, pool=big)
    b = agile.Mesh.from_workload(w)
    for x in (a, b):
        x.step_cfl(2)
    t0, dt0 = a.time(), a.last_dt()
    sa = a.regrid(refine, coarsen, 3, variable=4)
    sb = b.regrid(refine, coarsen, 3, variable=4)
    _say(f"regrid in a pool: {sa}")
    assert sa == sb and sa["refined"] > 0
    assert np.array_equal(a.blocks(), b.blocks())
    assert np.array_equal(a.readback(), b.readback())
    assert a.time() == t0 and a.last_dt() == dt0
    a.step_cfl(1)
    b.step_cfl(1)
    assert np.array_equal(a.readback(), b.readback())


def test_batch_in_a_torch_pool_equals_library_allocation(agile):
    import torch
    ws = [W.sedov(base_blocks=4, nlevels=3), W.uniform_random(nb=2, riemann=W.HLLC),
          W.smooth_random(W.refine_blocks(W.uniform_blocks((2, 2, 2)), [0]), (2, 2, 2), 2, seed=4)]
    pool = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    out = []
    for p in (pool, None):
        b = agile.Batch(riemann=W.HLLC, budget_bytes=256 << 20, pool=p)
        for tag, w in enumerate(ws):
            b.submit(w, 3, tag)
        for _ in range(3):
            b.tick()
        out.append([b.result(tag)[0] for tag in range(len(ws))])
        _say(f"batch pool={p is not None}: capacity {b.capacity()}")
        b.close()
    for tag in range(len(ws)):
        assert np.array_equal(out[0][tag], out[1][tag]), tag
