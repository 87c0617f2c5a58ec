"""Pins of the oracle's benchmark numerics of Sec. 3.1 (local Lax-Friedrichs
flux, van Leer limiter, three-stage SSP Runge-Kutta) against things other than
itself: the exact double-Sod solution, consistency and relative dissipation
of the fluxes, second-order convergence and accuracy relative to minmod,
temporal order of the integrators on a fixed grid, mirror symmetry and
conservation across level jumps.  CPU only."""
from __future__ import annotations

import math

import numpy as np
import pytest

from exact_riemann import double_sod_density
from oracle import oracle as orc
from oracle.oracle import Oracle
from paper_2607_19277_amd import workloads as W
from test_oracle import _mirror_check, line_profile, run_to, totals


def scheme(w, riemann=None, limiter=None, rk=None):
    if riemann is not None:
        w.riemann = riemann
    if limiter is not None:
        w.limiter = limiter
    if rk is not None:
        w.rk = rk
    return w


@pytest.fixture
def one_thread():
    n = orc.threads()
    orc.set_threads(1)
    yield
    orc.set_threads(n)


def _sod_errors(riemann, limiter, rk, ns=(128, 256, 512), t_end=0.1):
    errs = []
    for n in ns:
        w = scheme(W.double_sod(n, axis=0, riemann=riemann), limiter=limiter, rk=rk)
        o = Oracle(w)
        run_to(o, t_end)
        rho = line_profile(w, o.state())
        x = (np.arange(n) + 0.5) / n
        errs.append(float(np.abs(rho - double_sod_density(x, t_end)).mean()))
    return errs


def test_lf_vanleer_rk3_converges_to_exact_double_sod(one_thread):
    errs = _sod_errors(W.LF, W.VANLEER, 3)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 0.7 and errs[-1] < 8e-3, (errs, rates)


def test_lf_is_consistent_and_more_diffusive_than_hll(one_thread):
    w = W.double_sod(64, axis=0)
    o = Oracle(scheme(w, riemann=W.LF))
    h = Oracle(scheme(W.double_sod(64, axis=0), riemann=W.HLL))
    for wl in ([1.0, 0.3, -0.1, 0.2, 0.9], [0.4, -1.2, 0.0, 0.5, 0.05]):
        for d in range(3):
            a = o.face_flux(wl, wl, d)
            b = h.face_flux(wl, wl, d)
            assert np.allclose(a, b, rtol=1e-15, atol=1e-15)
    # on a jump the LF flux dissipates more: larger L1 error than HLL on the same grid
    e_lf = _sod_errors(W.LF, W.MINMOD, 2, ns=(256,))[0]
    e_hll = _sod_errors(W.HLL, W.MINMOD, 2, ns=(256,))[0]
    assert e_lf > 1.1 * e_hll, (e_lf, e_hll)


def _wave_error(n, riemann, limiter, rk, t_end=0.25):
    nb = n // 16
    w = W.density_wave(W.uniform_blocks((nb, 1, 1)), (nb, 1, 1), bn=(16, 2, 2), vel=(1.0, 0.0, 0.0), kvec=(1, 0, 0))
    scheme(w, riemann, limiter, rk)
    o = Oracle(w)
    run_to(o, t_end)
    x, _, _, _ = W.cell_coords(w.blocks, w.bn, w.base, w.lo, w.hi)
    ref = 1.0 + 0.2 * np.sin(2.0 * np.pi * (x - t_end))
    return float(np.abs(o.state()[:, 0] - ref).mean())


def test_vanleer_is_second_order_and_sharper_than_minmod(one_thread):
    ev = [_wave_error(n, W.LF, W.VANLEER, 3) for n in (32, 64, 128)]
    em = [_wave_error(n, W.LF, W.MINMOD, 3) for n in (32, 64, 128)]
    orders = [math.log2(ev[i] / ev[i + 1]) for i in range(2)]
    assert orders[-1] > 1.8, (ev, orders)
    assert all(a < b for a, b in zip(ev, em)), (ev, em)


@pytest.mark.parametrize("rk,lo,hi", [(2, 3.4, 4.6), (3, 6.5, 10.5)])
def test_time_integrator_order_on_a_fixed_grid(one_thread, rk, lo, hi):
    """Same grid and spatial operator, dt halved: the difference to a
    dt/16 run falls by 2^order (second order for SSP-RK2, third for SSP-RK3)."""
    def run(dt, nsteps):
        w = W.density_wave(W.uniform_blocks((4, 1, 1)), (4, 1, 1), bn=(16, 2, 2), vel=(1.0, 0.0, 0.0),
                           kvec=(1, 0, 0), amp=0.2)
        scheme(w, W.LF, W.VANLEER, rk)
        o = Oracle(w)
        for _ in range(nsteps):
            o.step(dt)
        return o.state()[:, 0]
    w0 = W.density_wave(W.uniform_blocks((4, 1, 1)), (4, 1, 1), bn=(16, 2, 2), vel=(1.0, 0.0, 0.0), kvec=(1, 0, 0))
    dt0 = 2.0 * Oracle(w0).dt()            # a CFL of about 0.8 along the tube
    ref = run(dt0 / 16, 128)
    e = [float(np.abs(run(dt0 / m, 8 * m) - ref).max()) for m in (1, 2, 4)]
    ratios = [e[i] / e[i + 1] for i in range(2)]
    assert lo < ratios[0] < hi and lo < ratios[1] < hi, (e, ratios)


@pytest.mark.parametrize("riemann,limiter", [(W.LF, W.VANLEER), (W.HLLC, W.VANLEER)])
def test_mirror_symmetry(one_thread, riemann, limiter):
    w = scheme(W.double_sod(128, axis=0, riemann=riemann), limiter=limiter, rk=3)
    o = Oracle(w)
    for _ in range(40):
        o.step(o.dt())
    _mirror_check(w, o.state(), 0)


def test_conservation_with_level_jumps():
    blocks, base, lmax = W.refine_blocks(W.uniform_blocks((2, 2, 2)), [0]), (2, 2, 2), 2
    w = scheme(W.smooth_random(blocks, base, lmax, seed=6), W.LF, W.VANLEER, 3)
    o = Oracle(w)
    t0 = totals(w, w.U)
    for _ in range(3):
        o.step(o.dt())
    t1 = totals(w, o.state())
    for (a, na), (b, nb) in zip(t0, t1):
        assert abs(b - a) <= 1e-14 * na, (a, b, na)
