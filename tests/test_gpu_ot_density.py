"""The Orszag-Tang mesh refined on the density (the benchmark's MHD
configuration), on an MHD box small enough for the oracle, through the C-ABI:
both sides advance the vortex on the base grid with their own CFL steps, then
regrid twice on the Loehner estimate of the density (thresholds in the widest
gap of the oracle's estimates near the benchmark's fractions, so that rounding
cannot move a block across them); the leaves equal the oracle's, the state is
within the FP64 bar, and so is the CFL step that follows."""
from __future__ import annotations

import dataclasses
import sys

import numpy as np
import pytest

from oracle import regrid as RG
from oracle.oracle import Oracle
from paper_2607_19277_amd import workloads as W
from parity import parity_error_mhd

pytestmark = pytest.mark.gpu
TOL = 1e-12
T_END = 0.05


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _gap_threshold(est, lev, frac):
    """A refine threshold near the (1 - frac) quantile of the finest level's
    estimates, in the widest gap between neighbouring values there."""
    fine = np.sort(est[lev == lev.max()])
    k = int(np.clip(round((1.0 - frac) * (len(fine) - 1)), 1, len(fine) - 1))
    lo, hi = max(1, k - 3), min(len(fine) - 1, k + 3)
    g = lo + int(np.argmax(np.diff(fine[lo - 1:hi + 1])[: hi - lo + 1]))
    return 0.5 * (fine[g - 1] + fine[g])


def test_density_refined_vortex_matches_oracle():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    from paper_2607_19277_amd import agile
    w = W.orszag_tang(base=(4, 4, 1), nlevels=3, blocks=W.uniform_blocks((4, 4, 1)))
    m = agile.Mesh.from_workload(w)
    o = Oracle(w)
    n = 0
    t_o = 0.0
    while t_o < T_END:
        dt = o.dt()
        o.step(dt)
        t_o += dt
        m.step_cfl(1)
        n += 1
    assert abs(m.time() - t_o) <= 1e-12 * t_o
    _say(f"{n} base-grid steps to t = {t_o:.4f}")
    blocks = np.asarray(w.blocks)
    for r, frac in enumerate((0.6, 0.5)):
        wr = dataclasses.replace(w, blocks=blocks, U=o.state())
        est = Oracle(wr).lohner(0, 0.01)
        e_gpu = m.error(0)
        assert np.max(np.abs(e_gpu - est)) <= 1e-9, np.max(np.abs(e_gpu - est))
        thr = _gap_threshold(est, blocks[:, 0], frac)
        new, R, P = RG.decide(blocks, est, w.base, r + 2, thr, -1.0)
        st = m.regrid(thr, -1.0, r + 2, variable=0)
        _say(f"regrid {r + 1}: threshold {thr:.4g}, {len(blocks)} -> {len(new)} blocks")
        assert [tuple(b) for b in m.blocks().tolist()] == new and st["refined"] == len(R) > 0
        U_new = Oracle(wr).remap(new)
        blocks = np.array(new, dtype=np.int32)
        o = Oracle(dataclasses.replace(w, blocks=blocks, U=U_new))
        err = parity_error_mhd(m.readback(), U_new, w.gamma).max()
        assert err <= TOL, err
    dt = o.dt()
    m.step_cfl(1)
    assert abs(m.last_dt() - dt) <= 1e-12 * dt
    o.step(dt)
    err = parity_error_mhd(m.readback(), o.state(), w.gamma)
    _say(f"step on the refined mesh ({len(blocks)} blocks, levels {sorted(set(blocks[:, 0].tolist()))}): "
         f"err {err.max():.2e}")
    assert err.max() <= TOL
