"""The benchmark numerics of Sec. 3.1 (local Lax-Friedrichs flux, van Leer
limiter, three-stage SSP Runge-Kutta) and their combinations with the other
solvers on an MI355X through the C-ABI, against the CPU oracle: one step from
the oracle's state to the FP64 bar, on meshes with and without level jumps."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2607_19277_amd import workloads as W
from parity import TOL_FP64, parity_error

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


MESHES = {
    "uniform": lambda: W.uniform_random(nb=2),
    "corner": lambda: W.smooth_random(W.refine_blocks(W.uniform_blocks((2, 2, 2)), [0]), (2, 2, 2), 2, seed=4),
    "dependent3": lambda: W.smooth_random(W.dependent_levels_blocks(), (4, 4, 4), 3, seed=17),
}
SCHEMES = {
    "lf_vanleer_rk3": (W.LF, W.VANLEER, 3),
    "lf_minmod_rk2": (W.LF, W.MINMOD, 2),
    "hllc_vanleer_rk3": (W.HLLC, W.VANLEER, 3),
    "hll_minmod_rk3": (W.HLL, W.MINMOD, 3),
}


def _with(w, sch):
    w.riemann, w.limiter, w.rk = sch
    return w


@pytest.mark.parametrize("mesh", list(MESHES))
@pytest.mark.parametrize("sch", list(SCHEMES))
def test_step_matches_oracle(agile, mesh, sch):
    w = _with(MESHES[mesh](), SCHEMES[sch])
    _say(f"{sch} on {mesh}: {w.nblocks} blocks")
    o = Oracle(w)
    m = agile.Mesh.from_workload(w)
    for s in range(2):
        m.set_blocks(w.blocks, o.state())
        dt = o.dt()
        assert m.dt() == dt
        m.step(dt)
        o.step(dt)
        err = parity_error(m.readback(), o.state(), w.gamma)
        _say(f"  step {s}: err {err.max():.3e}")
        assert err.max() <= TOL_FP64, err


def test_rk3_cfl_steps_equal_host_dt_steps(agile):
    w = _with(MESHES["dependent3"](), SCHEMES["lf_vanleer_rk3"])
    a = agile.Mesh.from_workload(w)
    b = agile.Mesh.from_workload(w)
    for _ in range(3):
        a.step(a.dt())
    b.step_cfl(3)
    assert np.array_equal(a.readback(), b.readback())


def test_fp32_flux_lf_vanleer_rk3_close_to_fp64(agile):
    w = _with(W.kelvin_helmholtz(n=64), SCHEMES["lf_vanleer_rk3"])
    a = agile.Mesh.from_workload(w)
    b = agile.Mesh.from_workload(w, precision=agile.FP32_FLUX)
    dt = a.dt()
    for _ in range(5):
        a.step(dt)
        b.step(dt)
    Ua, Ub = a.readback(), b.readback()
    scale = np.abs(Ua).max(axis=(0, 2, 3, 4))
    scale[1:4] = np.sqrt((Ua[:, 1:4] ** 2).sum(axis=1)).max()
    err = np.abs(Ua - Ub).max(axis=(0, 2, 3, 4)) / scale
    _say(f"fp32 vs fp64 (LF, van Leer, RK3) after 5 steps: {err}")
    assert err.max() < 1e-5


def test_batch_rejects_other_schemes(agile):
    w = _with(W.uniform_random(nb=2, riemann=W.HLLC), (W.HLLC, W.VANLEER, 3))
    b = agile.Batch(riemann=agile.HLLC)
    with pytest.raises(agile.AgileError):
        b.submit(w, 1, 1)
