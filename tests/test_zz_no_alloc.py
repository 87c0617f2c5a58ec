"""The regrid entry point that allocates no device memory
(agile_mesh_regrid_noalloc), through the C-ABI on an MI355X, against the
allocating agile_mesh_regrid on identical meshes: two calls in a row on one
GPU, the second on a smaller mesh (it shares the first call's static task
table), each giving the same leaves, bitwise the same state, time and dt, and
the same next step.  A regrid whose new mesh does not fit is refused and
leaves the mesh as it was."""
from __future__ import annotations

import dataclasses
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
                      max_level=w.max_level)["device_bytes"]


def _compare(agile, a, b, w, refine, coarsen, variable):
    """a: regrid without allocation, b: the allocating regrid; both from the
    same state."""
    for x in (a, b):
        x.step_cfl(2)
    t0, dt0 = a.time(), a.last_dt()
    sa = a.regrid_noalloc(refine, coarsen, w.max_level, variable=variable)
    sb = b.regrid(refine, coarsen, w.max_level, variable=variable)
    _say(f"  no-alloc {sa}, allocating {sb}")
    assert sa == sb
    assert np.array_equal(a.blocks(), b.blocks())
    assert np.array_equal(a.readback(), b.readback())
    assert a.time() == t0 == b.time() and a.last_dt() == dt0 == b.last_dt()
    a.step_cfl(1)
    b.step_cfl(1)
    assert np.array_equal(a.readback(), b.readback())
    assert a.last_dt() == b.last_dt()
    return sa


def test_two_regrids_in_a_row_equal_the_allocating_regrid(agile):
    import torch
    # call 1: a refining regrid of a 3-level mesh in a caller pool with room to grow
    w1 = dataclasses.replace(W.sedov(base_blocks=4, nlevels=3), max_level=4)
    pool = torch.empty(4 * _need(agile, w1), dtype=torch.uint8, device="cuda")
    a1 = agile.Mesh.from_workload(w1, pool=pool)
    b1 = agile.Mesh.from_workload(w1)
    _say(f"call 1: sedov3, {w1.nblocks} blocks")
    s1 = _compare(agile, a1, b1, w1, refine=0.5, coarsen=-1.0, variable=4)
    assert s1["refined"] > 0 and s1["new_blocks"] > w1.nblocks
    # call 2: a smaller, library-allocated mesh whose regrid coarsens (it fits)
    w2 = W.smooth_random(W.refine_blocks(W.uniform_blocks((2, 2, 2)), [0]), (2, 2, 2), 2, seed=4)
    a2 = agile.Mesh.from_workload(w2)
    b2 = agile.Mesh.from_workload(w2)
    _say(f"call 2: corner mesh, {w2.nblocks} blocks")
    s2 = _compare(agile, a2, b2, w2, refine=2.0, coarsen=1.5, variable=4)
    assert s2["coarsened"] == 1 and s2["new_blocks"] == 8 < s1["new_blocks"]
    for x in (a1, b1, a2, b2):
        x.close()


def test_regrid_that_does_not_fit_is_refused(agile):
    """A library-allocated mesh has no room to grow: a refining regrid without
    allocation returns AGILE_ENOMEM (not sticky) and the mesh steps on."""
    w = dataclasses.replace(W.smooth_random(W.nested_blocks((4, 4, 4), 2), (4, 4, 4), 2, seed=21), max_level=3)
    m = agile.Mesh.from_workload(w)
    m.step_cfl(1)
    before = m.readback()
    with pytest.raises(agile.AgileError) as e:
        m.regrid_noalloc(0.0, -1.0, 3, variable=4)      # refine every block
    assert e.value.code == agile.ENOMEM
    assert np.array_equal(m.readback(), before)
    assert np.array_equal(m.blocks(), np.asarray(w.blocks))
    m.step_cfl(1)
    m.close()
