"""Full-size parity on an MI355X: the Sedov blast mesh (128^3 base, 3 nested
2:1 levels, 1856 leaves, HLLC) and the 256^3 Kelvin-Helmholtz box (4096
blocks), each in the launch configuration the benchmark times (default stage
shape, CFL dt reduced on the device), against the CPU oracle on the whole
state.  Ghosts and dt bitwise, the state to the FP64 bar."""
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


def _full_step(agile, w, ghosts):
    _say(f"{w.name}: {w.nblocks} blocks, {w.ncells} cells")
    o = Oracle(w)
    m = agile.Mesh.from_workload(w)
    if ghosts:
        g = m.read_ghosts()
        ref = o.ghosts()
        bad = np.argwhere(g != ref)
        assert bad.size == 0, bad[:5]
        del g, ref
        _say("  ghost fill bitwise equal")
    dt = o.dt()
    assert m.dt() == dt
    m.step_cfl(1)                      # dt from the device reduction, as in the timed steps
    assert m.last_dt() == dt
    o.step(dt)
    Ug = m.readback()
    err = parity_error(Ug, o.state(), w.gamma)
    _say(f"  one step, dt={dt:.6e}: err per var {np.array2string(err, precision=2)}")
    assert err.max() <= TOL_FP64, err
    # next dt from the signal maximum fused into stage 2: bitwise the oracle's
    # dt of the same (device) state, and within the state bar of the oracle's own
    d_next = m.dt()
    assert d_next == Oracle(w, U=Ug).dt()
    assert abs(d_next - o.dt()) <= TOL_FP64 * o.dt()
    m.close()


def test_sedov_full_size(agile):
    _full_step(agile, W.sedov(base_blocks=8, nlevels=4, riemann=W.HLLC), ghosts=True)


def test_kelvin_helmholtz_256(agile):
    _full_step(agile, W.kelvin_helmholtz(n=256), ghosts=False)


def test_orszag_tang_full_size(agile):
    """Ideal MHD + GLM on the 4-level Orszag-Tang mesh (18 944 leaves, 77.6 M
    cells): one CFL step from the device reduction against the oracle."""
    from parity import parity_error_mhd
    w = W.orszag_tang()
    _say(f"{w.name}: {w.nblocks} blocks, {w.ncells} cells")
    o = Oracle(w)
    m = agile.Mesh.from_workload(w)
    dt = o.dt()
    assert m.dt() == dt
    m.step_cfl(1)
    assert m.last_dt() == dt
    o.step(dt)
    err = parity_error_mhd(m.readback(), o.state(), w.gamma)
    _say(f"  one step, dt={dt:.6e}: err per var {np.array2string(err, precision=2)}")
    assert err.max() <= TOL_FP64, err
    m.close()


def test_kelvin_helmholtz_256_paper_numerics(agile):
    """The benchmark numerics of Sec. 3.1 (LF, van Leer, SSP-RK3) on the 256^3
    shear layer: one CFL step against the oracle."""
    w = W.kelvin_helmholtz(n=256)
    w.riemann, w.limiter, w.rk = W.LF, W.VANLEER, 3
    _full_step(agile, w, ghosts=False)
