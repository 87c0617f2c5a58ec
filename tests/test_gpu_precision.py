"""Mixed precision (FP32 reconstruction and Riemann flux, FP64 state,
divergence accumulation, flux correction and dt) against the FP64 oracle:
the Kelvin-Helmholtz shear layer run to t = 0.5 on a 64^3 box, every side with
its own CFL steps.  The relative L1 error of density and total energy must
stay within 1e-5; the FP64 path is reported beside it."""
from __future__ import annotations

import sys

import pytest

import kh_l1
from paper_2607_19277_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_kh64_to_half_l1_against_oracle():
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    w = W.kelvin_helmholtz(n=64)
    R, t_ref, n_ref = kh_l1.oracle_run(w)
    print(f"oracle: {n_ref} steps to t={t_ref}", flush=True)
    out = {}
    for prec, name in ((0, "fp64"), (1, "fp32flux")):
        U, t, n = kh_l1.gpu_run(w, prec)
        out[name] = (kh_l1.l1_rel(U[:, 0], R[:, 0]), kh_l1.l1_rel(U[:, 4], R[:, 4]))
        print(f"{name}: {n} steps to t={t}; L1 rel rho {out[name][0]:.3e}, e {out[name][1]:.3e}", flush=True)
        sys.stdout.flush()
        assert abs(t - t_ref) < 1e-12
    assert max(out["fp32flux"]) <= 1e-5
    assert max(out["fp64"]) <= 1e-9


def test_srhd_shear_layer_64_to_half_l1_against_oracle():
    """The same check for the relativistic shear layer (LF, van Leer, SSP-RK3,
    the numerics of the SRHD benchmark) on a 64^3 box: the FP32-flux path
    within 1e-5 in relative L1 of D and tau at t = 0.5."""
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    w = W.srhd_kelvin_helmholtz(n=64)
    w.limiter, w.rk = W.VANLEER, 3
    R, t_ref, n_ref = kh_l1.oracle_run(w)
    print(f"oracle: {n_ref} steps to t={t_ref}", flush=True)
    out = {}
    for prec, name in ((0, "fp64"), (1, "fp32flux")):
        U, t, n = kh_l1.gpu_run(w, prec)
        out[name] = (kh_l1.l1_rel(U[:, 0], R[:, 0]), kh_l1.l1_rel(U[:, 4], R[:, 4]))
        print(f"srhd {name}: {n} steps to t={t}; L1 rel D {out[name][0]:.3e}, tau {out[name][1]:.3e}", flush=True)
        sys.stdout.flush()
        assert abs(t - t_ref) < 1e-12
    assert max(out["fp32flux"]) <= 1e-5
    assert max(out["fp64"]) <= 1e-9
