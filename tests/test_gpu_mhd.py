"""Ideal MHD + GLM (Sec. 2.3.3) on an MI355X through the C-ABI against the
CPU oracle: ghost fill of all nine variables bitwise, dt (fast speeds)
bitwise, one step from the oracle's state to the FP64 bar
(tests/parity.py, MHD metric), conservation and the FP32-flux form."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2607_19277_amd import workloads as W
from parity import TOL_FP64, parity_error_mhd

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


CASES = {
    "uniform": lambda: W.mhd_smooth_random(W.uniform_blocks((2, 2, 2)), (2, 2, 2), 1, seed=4, psi_amp=0.05),
    "corner": lambda: W.mhd_smooth_random(W.refine_blocks(W.uniform_blocks((2, 2, 2)), [0]), (2, 2, 2), 2, seed=8,
                                          psi_amp=0.05),
    "nested3": lambda: W.mhd_smooth_random(W.nested_blocks((4, 4, 4), 3), (4, 4, 4), 3, seed=12, b_amp=0.8),
    "alfven": lambda: W.alfven_wave(64, bn_long=16, bn_short=16),
}


@pytest.mark.parametrize("case", list(CASES))
def test_mhd_ghosts_and_dt_bitwise(agile, case):
    w = CASES[case]()
    _say(f"mhd ghosts/dt {case}: {w.nblocks} blocks")
    m = agile.Mesh.from_workload(w)
    o = Oracle(w)
    g, ref = m.read_ghosts(), o.ghosts()
    bad = np.argwhere(g != ref)
    assert bad.size == 0, bad[:5]
    assert m.dt() == o.dt()


@pytest.mark.parametrize("case", list(CASES))
def test_mhd_step_matches_oracle(agile, case):
    w = CASES[case]()
    _say(f"mhd step {case}")
    o = Oracle(w)
    m = agile.Mesh.from_workload(w)
    for s in range(3):
        m.set_blocks(w.blocks, o.state())
        dt = o.dt()
        m.step(dt)
        o.step(dt)
        err = parity_error_mhd(m.readback(), o.state(), w.gamma)
        _say(f"  step {s}: dt={dt:.6e} err={err.max():.3e} per-var={np.array2string(err, precision=2)}")
        assert err.max() <= TOL_FP64, (s, err)


def test_mhd_step_cfl_equals_host_dt_step(agile):
    w = CASES["corner"]()
    a = agile.Mesh.from_workload(w)
    b = agile.Mesh.from_workload(w)
    for _ in range(3):
        a.step(a.dt())
    b.step_cfl(3)
    assert np.array_equal(a.readback(), b.readback())
    assert a.last_dt() == b.last_dt()


def test_mhd_conservation_on_gpu(agile):
    w = CASES["nested3"]()
    m = agile.Mesh.from_workload(w)
    m.step_cfl(4)
    U = m.readback()
    vol = np.array([w.dx(int(l)) ** 3 for l in w.blocks[:, 0]])[:, None]
    for v in range(8):
        a = (w.U[:, v].reshape(w.nblocks, -1) * vol).sum()
        b = (U[:, v].reshape(w.nblocks, -1) * vol).sum()
        n = (np.abs(w.U[:, v]).reshape(w.nblocks, -1) * vol).sum()
        assert abs(b - a) <= 1e-13 * n, (v, a, b)


def test_mhd_fp32_flux_close_to_fp64(agile):
    w = CASES["nested3"]()
    a = agile.Mesh.from_workload(w)
    b = agile.Mesh.from_workload(w, precision=agile.FP32_FLUX)
    dt = a.dt()
    for _ in range(4):
        a.step(dt)
        b.step(dt)
    Ua, Ub = a.readback(), b.readback()
    scale = np.abs(Ua).max(axis=(0, 2, 3, 4))
    # psi grows from the divergence error only: measure it on its natural
    # scale, the fast speed times |B|
    bb = (Ua[:, 5:8] ** 2).sum(axis=1)
    p = (w.gamma - 1.0) * (Ua[:, 4] - 0.5 * (Ua[:, 1:4] ** 2).sum(axis=1) / Ua[:, 0] - 0.5 * bb)
    scale[8] = float(np.sqrt((w.gamma * p + bb) / Ua[:, 0]).max() * np.sqrt(bb).max())
    err = np.abs(Ua - Ub).max(axis=(0, 2, 3, 4)) / scale
    _say(f"mhd fp32 vs fp64 after 4 steps: {np.array2string(err, precision=2)}")
    assert err.max() < 1e-5
