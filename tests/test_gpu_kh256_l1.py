"""The Kelvin-Helmholtz shear layer of 256^3 cells in 16^3 blocks (HLLC,
minmod, SSP-RK2) run to t = 0.5 on an MI355X through the C-ABI, in FP64 and
in the FP32-flux form, against the FP64 oracle's own run of the same problem
(stored in tests/golden/kh256_t05_oracle_stride64.npz by
`python tests/kh_l1.py reference --n 256 --block-stride 64 --out ...`, which
calls the oracle only: about 2.7 h of host time).  Each side takes the CFL dt
of its own state and clips the last step to t = 0.5.  The stored density and
energy are float64, every 64th block of the block order (the x = 0 column at
every fourth y and every z, crossing both shear layers).

Bars: FP64 1e-12 relative L1 (the per-step parity bar; the two runs agree to
round-off), FP32 flux 1e-5 relative L1 (the mixed-precision bar)."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from kh_l1 import gpu_run, l1_rel  # noqa: E402

pytestmark = pytest.mark.gpu

REF = os.path.join(HERE, "golden", "kh256_t05_oracle_stride64.npz")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision,bar", [(0, 1e-12), (1, 1e-5)])
def test_kh256_to_t05_against_the_stored_oracle_run(precision, bar):
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    from paper_2607_19277_amd import agile, workloads as W
    agile.lib()
    R = np.load(REF)
    assert int(R["n"]) == 256 and str(R["physics"]) == "euler"
    stride = int(R["block_stride"])
    w = W.kelvin_helmholtz(n=256)
    U, t, n = gpu_run(w, precision)
    assert abs(t - 0.5) <= 1e-12 and abs(float(R["t"]) - 0.5) <= 1e-12
    sel = slice(None, None, stride)
    e_rho, e_e = l1_rel(U[sel, 0], R["rho"]), l1_rel(U[sel, 4], R["e"])
    _say(f"precision {precision}: {n} steps (oracle {int(R['steps'])}), L1 rho {e_rho:.3e}, e {e_e:.3e}")
    if precision == 0:
        assert n == int(R["steps"])
    assert e_rho <= bar and e_e <= bar
