"""Blocks of 32^3 and 64^3 cells (the other block sizes of the paper's
single-device study, Sec. 3.1, Table 4) on an MI355X through the C-ABI.  The
oracle runs these block sizes natively; the device stores a block as 16^3
tiles.  Checked: one step and consecutive CFL steps against the oracle to the
FP64 bar on uniform and two-level meshes, the same cell values as the same
mesh in 16^3 blocks (bitwise), and a regrid of 32^3 blocks (estimate and
transfer bitwise, the decision equal to the oracle's, the next step to the
bar)."""
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


def to_tiles(w):
    """The same cells as a mesh of 16^3 blocks: each block's sub-tiles in
    (z, y, x) order, the state cut accordingly."""
    te = w.bn[0] // 16
    n = w.nblocks
    U = w.U.reshape(n, w.nvar, te, 16, te, 16, te, 16).transpose(0, 2, 4, 6, 1, 3, 5, 7)
    U = np.ascontiguousarray(U.reshape(n * te ** 3, w.nvar, 16, 16, 16))
    b = []
    for (l, x, y, z) in w.blocks.tolist():
        for tz in range(te):
            for ty in range(te):
                for tx in range(te):
                    b.append((l, te * x + tx, te * y + ty, te * z + tz))
    base = tuple(te * c for c in w.base)
    return dataclasses.replace(w, bn=(16, 16, 16), base=base, blocks=np.array(b, dtype=np.int32), U=U)


CASES = {
    "kh64_b32": lambda: W.kelvin_helmholtz(n=64, bn=32),
    "corner_b32": lambda: W.smooth_random(W.refine_blocks(W.uniform_blocks((2, 2, 2)), [0]), (2, 2, 2), 2, seed=11, bn=32),
    "uniform128_b64": lambda: W.kelvin_helmholtz(n=128, bn=64),
}


@pytest.mark.parametrize("case", list(CASES))
def test_one_step_matches_oracle_and_16_blocks(agile, case):
    w = CASES[case]()
    _say(f"{case}: {w.nblocks} blocks of {w.bn[0]}^3")
    o = Oracle(w)
    dt = o.dt()
    m = agile.Mesh.from_workload(w)
    assert m.dt() == dt
    m.step(dt)
    U = m.readback()
    o.step(dt)
    err = parity_error(U, o.state(), w.gamma).max()
    _say(f"  one step: err {err:.2e}")
    assert err <= TOL_FP64
    t = agile.Mesh.from_workload(to_tiles(w))
    t.step(dt)
    assert np.array_equal(t.readback(), to_tiles(dataclasses.replace(w, U=U)).U)
    m.close()
    t.close()


def test_consecutive_cfl_steps_of_32_blocks(agile):
    w = CASES["corner_b32"]()
    R, t_ref = oracle_cfl_steps(w, 3)
    m = agile.Mesh.from_workload(w)
    m.step_cfl(3)
    err = parity_error(m.readback(), R, w.gamma).max()
    _say(f"three CFL steps: err {err:.2e}")
    assert err <= TOL_FP64 and abs(m.time() - t_ref) <= 1e-12 * t_ref


def test_regrid_of_32_blocks(agile):
    w = dataclasses.replace(CASES["corner_b32"](), max_level=3)
    m = agile.Mesh.from_workload(w)
    est = m.error(4)
    assert np.array_equal(est, Oracle(w).lohner(4, 0.01))
    refine, coarsen = float(np.quantile(est, 0.8)), float(np.quantile(est, 0.3))
    new_ref, R, P = RG.decide(w.blocks, est, w.base, w.max_level, refine, coarsen)
    st = m.regrid(refine, coarsen, w.max_level, variable=4)
    _say(f"regrid of 32^3 blocks: {st}")
    assert st["new_blocks"] == len(new_ref) and st["refined"] == len(R)
    assert [tuple(r) for r in m.blocks().tolist()] == new_ref
    U_ref = Oracle(w).remap(new_ref)
    assert np.array_equal(m.readback(), U_ref)
    w2 = dataclasses.replace(w, blocks=np.array(new_ref, dtype=np.int32), U=U_ref)
    o2 = Oracle(w2)
    dt = o2.dt()
    assert m.dt() == dt
    m.step(dt)
    o2.step(dt)
    assert parity_error(m.readback(), o2.state(), w.gamma).max() <= TOL_FP64
