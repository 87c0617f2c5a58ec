"""Pins of the oracle's special relativistic hydrodynamics (SRHD) module
against things other than itself: the numpy primitive -> conserved map of
the input generator (con2prim round trip), the flux Jacobian's eigenvalues,
the CFL closed form, the Newtonian limit (the Euler oracle), the exact
solution of an advected density wave, Newton's step count, conservation across level jumps and
mirror symmetry.  CPU only."""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import pytest

from oracle import oracle as orc
from oracle.oracle import Oracle
from paper_2607_19277_amd import workloads as W
from test_oracle import _mirror_check, line_profile, run_to, totals


@pytest.fixture
def one_thread():
    n = orc.threads()
    orc.set_threads(1)
    yield
    orc.set_threads(n)


def _srhd_oracle(gamma=5.0 / 3.0):
    w = W.srhd_smooth_random(W.uniform_blocks((1, 1, 1)), (1, 1, 1), 1, gamma=gamma)
    return Oracle(w), w


def test_con2prim_round_trip_over_a_range_of_states():
    o, _ = _srhd_oracle()
    rows = []
    for rho in (1e-2, 1.0, 1e2):
        for v in (0.0, 0.5, 0.9, 0.99, 0.999):
            for p in (1e-3, 1.0, 1e2):
                for ang in (0.3, 1.1):
                    vel = v * np.array([math.cos(ang), math.sin(ang) * 0.6, math.sin(ang) * 0.8])
                    rows.append((rho, *vel, p))
    P = np.array(rows)
    U = W.srhd_prim_to_cons(5.0 / 3.0, *(P[:, c].reshape(-1, 1) for c in range(5)))[:, :, 0]
    w = o.cons_to_prim(U)
    G = 1.0 / np.sqrt(1.0 - (P[:, 1:4] ** 2).sum(axis=1))
    ref = np.column_stack([P[:, 0], G[:, None] * P[:, 1:4], P[:, 4]])
    scale = np.column_stack([ref[:, 0], np.maximum(np.abs(ref[:, 1:4]), G[:, None]), ref[:, 4]])
    err = np.abs(w - ref) / scale
    # p = (g-1)/g (xi/Gamma^2 - rho) cancels when p/rho is small and Gamma
    # large (rho = 100, p = 1e-3, Gamma = 22: about 6e-9); elsewhere 1e-11
    assert err.max() < 1e-8, (err.max(), P[np.argmax(err.max(axis=1))])
    good = (P[:, 4] / P[:, 0] >= 1e-2) & (G <= 10)
    assert err[good].max() < 1e-11, err[good].max()


def test_newton_converges_quadratically_and_stops_on_an_exact_root():
    """At rest (m = 0) f is linear in xi, so the first Newton step from xi = e
    lands on the root and the second confirms it; on moving smooth states the
    quadratic convergence of Newton from xi = e reaches 1e-15 within a few
    steps.  A step that ends on a bracket end must count as converged, not
    restart bisection (which takes about 50 halvings to reach 1e-15)."""
    o, _ = _srhd_oracle(4.0 / 3.0)
    rest = W.srhd_prim_to_cons(4.0 / 3.0, np.array([[1.0, 1.0, 0.3]]), *(np.zeros((1, 3)),) * 3,
                               np.array([[100.0, 0.1, 1e-3]]))[:, :, 0]
    assert o.srhd_newton_steps(rest).max() <= 3
    w = W.srhd_smooth_random(W.uniform_blocks((2, 2, 2)), (2, 2, 2), 1, seed=3)
    U = np.moveaxis(w.U, 1, -1).reshape(-1, 5)
    steps = Oracle(w).srhd_newton_steps(U)
    assert steps.min() >= 2 and steps.max() <= 8, np.bincount(steps)


def _flux(o, U, d):
    w = o.cons_to_prim(U[None, :])[0]
    return o.face_flux(w, w, d)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_flux_jacobian_eigenvalues_are_the_characteristic_speeds(d):
    """The eigenvalues of dF/dU (central differences through con2prim) are
    lambda-, v_d (three times) and lambda+ of the textbook formula."""
    g = 5.0 / 3.0
    o, _ = _srhd_oracle(g)
    rho, p = 1.3, 0.7
    vel = np.array([0.45, -0.3, 0.25])
    U0 = W.srhd_prim_to_cons(g, np.array([[rho]]), *(np.array([[c]]) for c in vel), np.array([[p]]))[0, :, 0]
    J = np.zeros((5, 5))
    for k in range(5):
        h = 1e-6 * max(1.0, abs(U0[k]))
        Up, Um = U0.copy(), U0.copy()
        Up[k] += h
        Um[k] -= h
        J[:, k] = (_flux(o, Up, d) - _flux(o, Um, d)) / (2 * h)
    ev = np.sort(np.linalg.eigvals(J).real)
    v2 = (vel ** 2).sum()
    hh = 1.0 + g / (g - 1.0) * p / rho
    cs2 = g * p / (rho * hh)
    vd = vel[d]
    root = math.sqrt(cs2) * math.sqrt((1 - v2) * (1 - v2 * cs2 - vd * vd * (1 - cs2)))
    lam = sorted([(vd * (1 - cs2) - root) / (1 - v2 * cs2), vd, vd, vd, (vd * (1 - cs2) + root) / (1 - v2 * cs2)])
    assert np.allclose(ev, lam, atol=1e-6), (ev, lam)


def test_cfl_dt_closed_form():
    g = 4.0 / 3.0
    rho, vel, p = 0.8, np.array([0.6, 0.1, -0.2]), 2.0
    w = W.srhd_smooth_random(W.uniform_blocks((1, 1, 1)), (1, 1, 1), 1, gamma=g)
    w = dataclasses.replace(w, U=np.broadcast_to(
        W.srhd_prim_to_cons(g, np.array([[rho]]), *(np.array([[c]]) for c in vel), np.array([[p]]))[:, :, :1, None, None],
        (1, 5, 16, 16, 16)).copy())
    v2 = (vel ** 2).sum()
    cs2 = g * p / (rho * (1.0 + g / (g - 1.0) * p / rho))
    s = 0.0
    for d in range(3):
        vd = vel[d]
        a = (abs(vd) * (1 - cs2) + math.sqrt(cs2) * math.sqrt((1 - v2) * (1 - v2 * cs2 - vd * vd * (1 - cs2)))) / (1 - v2 * cs2)
        s += a / w.dx(1)
    assert abs(Oracle(w).dt() - w.cfl / s) <= 1e-13 * w.cfl / s


def test_newtonian_limit_matches_the_euler_oracle():
    """Slow, cold flow (|v| ~ 1e-3, p/rho ~ 1e-6): the SRHD right-hand side
    equals the Euler one (LF both) to O(v^2, p/rho).  On one level: at a level
    jump the SRHD ghosts interpolate primitives, the Euler ones conserved
    variables, which differ at second order in the cell size."""
    g = 5.0 / 3.0
    blocks = W.uniform_blocks((4, 4, 4))

    def prim(x, y, z, gi, lev):
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
        vx = 1e-3 * np.sin(2 * np.pi * (y + z))
        vy = 1e-3 * np.cos(2 * np.pi * (x - z))
        vz = 5e-4 * np.sin(2 * np.pi * (x + y))
        p = 1e-6 * (1.0 + 0.3 * np.sin(2 * np.pi * z))
        return rho, vx, vy, vz, p
    ws = W._make("srhd_cold", W.SRHD, W.LF, g, 0.4, blocks, (16, 16, 16), (4, 4, 4), (0, 0, 0), (1, 1, 1), 1, prim)
    we = W._make("euler_cold", W.EULER, W.LF, g, 0.4, blocks, (16, 16, 16), (4, 4, 4), (0, 0, 0), (1, 1, 1), 1, prim)
    Ls, Le = Oracle(ws).rhs(), Oracle(we).rhs()
    for v in range(5):
        scale = np.abs(Le[:, v]).max()
        assert np.abs(Ls[:, v] - Le[:, v]).max() <= 1e-3 * scale, (v, np.abs(Ls[:, v] - Le[:, v]).max(), scale)


def _adv_error(n, limiter, rk, t_end=0.25, v=0.6):
    w = dataclasses.replace(W.srhd_advection(n, v=v), limiter=limiter, rk=rk)
    o = Oracle(w)
    run_to(o, t_end)
    rho = line_profile(w, o.state()) / (1.0 / math.sqrt(1 - v * v))     # D / Gamma
    x = (np.arange(n) + 0.5) / n
    return float(np.abs(rho - (1.0 + 0.3 * np.sin(2 * np.pi * (x - v * t_end)))).mean())


@pytest.mark.parametrize("limiter,rk,lo", [(W.VANLEER, 3, 1.8), (W.MINMOD, 2, 1.4)])
def test_advected_density_wave_converges(one_thread, limiter, rk, lo):
    errs = [_adv_error(n, limiter, rk) for n in (64, 128, 256)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[-1] > lo and errs[-1] < 5e-4, (errs, rates)


def test_conservation_with_level_jumps_and_mirror_symmetry():
    blocks = W.nested_blocks((4, 4, 4), 2)
    w = W.srhd_smooth_random(blocks, (4, 4, 4), 2)
    o = Oracle(w)
    t0 = totals(w, o.state())
    for _ in range(3):
        o.step(o.dt())
    t1 = totals(w, o.state())
    for (a, sa), (b, _) in zip(t0, t1):
        assert abs(a - b) <= 1e-13 * sa, (a, b)

    wb = W.srhd_blast(blocks)
    ob = Oracle(wb)
    for _ in range(15):
        ob.step(ob.dt())
    U = ob.state()
    for axis in range(3):
        _mirror_check(wb, U, axis)
    # the blast drives Lorentz factors above 1.2
    wv = ob.cons_to_prim(np.moveaxis(U, 1, -1).reshape(-1, 5))
    assert np.sqrt(1 + (wv[:, 1:4] ** 2).sum(axis=1)).max() > 1.2


def _srhd_cons(g, rho, u, p):
    """(D, m, tau) from rho, the four-velocity u (3 arrays) and p, written out
    from the SRHD definitions (Sec. 2.3.4), independently of the oracle."""
    G = np.sqrt(1.0 + (u[0] ** 2 + u[1] ** 2 + u[2] ** 2))
    rhoh = rho + g / (g - 1.0) * p
    return np.stack([G * rho, G * rhoh * u[0], G * rhoh * u[1], G * rhoh * u[2], G * G * rhoh - p - G * rho])


def test_prolongation_interpolates_the_primitives():
    """With rho, u = Gamma v and p linear in y and z only, every x-face ghost
    of a finer block next to a coarser one (limited linear prolongation)
    holds the conserved state of the exact primitives at its centre: the
    tangential slopes come from coarse leaves, and the normal slope is zero
    (its outer difference vanishes, so minmod gives 0 whatever the restricted
    inner neighbour holds).  Interpolating the conserved variables instead
    misses by the curvature of the primitive -> conserved map, ~1e-6."""
    from test_oracle import ghost_centres
    g = 4.0 / 3.0
    a = (1.0, 0.3, -0.2, 0.1, 2.0)
    b = ((-0.25, 0.75), (0.1, -0.1), (-0.2, 0.15), (0.1, 0.2), (0.25, -0.5))

    def lin(v, y, z):
        return a[v] + b[v][0] * y + b[v][1] * z

    def prim(x, y, z, gl, lev):
        u = [lin(1 + d, y, z) for d in range(3)]
        G = np.sqrt(1.0 + (u[0] ** 2 + u[1] ** 2 + u[2] ** 2))
        return (lin(0, y, z), u[0] / G, u[1] / G, u[2] / G, lin(4, y, z))
    blocks = W.nested_blocks((4, 4, 4), 2)
    w = W._make("srhd_linear", W.SRHD, W.LF, g, 0.4, blocks, (16, 16, 16), (4, 4, 4), (0, 0, 0), (1, 1, 1), 2, prim)
    gh = Oracle(w).ghosts()
    checked = 0
    for q, (l, ix, iy, iz) in enumerate(blocks.tolist()):
        if l != 2 or not (4 <= iy < 12 and 4 <= iz < 12):
            continue
        for f in (0, 1):
            nbx = ix + (1 if f else -1)
            if 4 <= nbx < 12:
                continue                      # a same-level neighbour: a copy
            x, y, z, _, _, _ = ghost_centres(w, q, f)
            ref = _srhd_cons(g, lin(0, y, z), [lin(1 + e, y, z) for e in range(3)], lin(4, y, z))
            got = gh[q, f].reshape(5, -1)
            assert np.abs(got - ref).max() <= 4e-14 * np.abs(ref).max(), (q, f, np.abs(got - ref).max())
            checked += 1
    assert checked >= 16, checked


def test_refining_across_a_relativistic_shock_stays_physical():
    """The relativistic blast after three steps, refined where Loehner's
    estimate of D is large: every new cell has a physical state (prolonged
    conserved variables give |m| > tau + D in 8 of the new blocks)."""
    import dataclasses
    from oracle import regrid as RG
    w = dataclasses.replace(W.srhd_blast(), max_level=3)
    o = Oracle(w)
    for _ in range(3):
        o.step(o.dt())
    w1 = dataclasses.replace(w, U=o.state())
    err = Oracle(w1).lohner(0, 0.01)
    new, R, _ = RG.decide(w.blocks, err, w.base, w.max_level, float(np.quantile(err, 0.85)),
                          float(np.quantile(err, 0.3)))
    assert len(R) >= 8
    U = Oracle(w1).remap(new)
    P = o.cons_to_prim(np.moveaxis(U, 1, -1).reshape(-1, 5))
    assert (P[:, 0] > 0).all() and (P[:, 4] > 0).all()


def test_exact_riemann_solver_satisfies_jump_conditions_and_newtonian_limit():
    """The exact SRHD Riemann solver used below, checked against things other
    than itself: across each shock it returns, the conserved fluxes jump by
    the shock speed times the conserved jump (Rankine-Hugoniot); with
    p/rho ~ 1e-6 its star state is the Newtonian one (Sod, exact Euler
    solver) to O(p/rho)."""
    import exact_riemann as E
    import exact_srhd_riemann as X
    g = 4.0 / 3.0

    def cons_flux(rho, v, p):
        W_ = 1.0 / math.sqrt(1.0 - v * v)
        rh = rho * X.enthalpy(rho, p, g)
        D, S, tau = rho * W_, rh * W_ * W_ * v, rh * W_ * W_ - p - rho * W_
        return np.array([D, S, tau]), np.array([D * v, S * v + p, S - D * v])
    for a, p, s in (((1.0, 0.2, 0.1), 5.0, 1), ((1.0, 0.2, 0.1), 5.0, -1), ((2.0, -0.5, 1.0), 30.0, 1),
                    ((0.5, 0.9, 0.01), 2.0, -1)):
        v, rho, Vs = X.shock(a, p, g, s)
        Ua, Fa = cons_flux(*a)
        Ub, Fb = cons_flux(rho, v, p)
        assert np.abs(Fb - Fa - Vs * (Ub - Ua)).max() <= 1e-14 * np.abs(Fb).max(), (a, p, s)
    eps = 1e-6
    ps, vs = X.star_state((1.0, 0.0, eps), (0.125, 0.0, 0.1 * eps), 1.4)
    pe, ue = E.star_state((1.0, 0.0, eps), (0.125, 0.0, 0.1 * eps), 1.4)
    assert abs(ps / pe - 1.0) < 1e-5 and abs(vs / ue - 1.0) < 1e-5, (ps / pe - 1.0, vs / ue - 1.0)


@pytest.mark.parametrize("limiter,rk", [(W.MINMOD, 2), (W.VANLEER, 3)])
def test_relativistic_double_shock_tube_converges_to_exact_solution(limiter, rk):
    """Periodic double tube (rho = 1 at rest, p = 10 in [1/4, 3/4], 0.1
    outside, g = 4/3; v* = 0.66, a dense shell of rho 5.5 behind a shock at
    0.8): the density converges in L1 to the exact solution at t = 0.2 (the
    shell is 17 cells wide at 512 cells, so the rate grows with resolution)
    and the shock sits within 3 cells of its exact position."""
    import exact_srhd_riemann as X
    g, t_end = 4.0 / 3.0, 0.2
    inside, outside = (1.0, 0.0, 10.0), (1.0, 0.0, 0.1)
    errs = []
    for n in (128, 256, 512):
        w = dataclasses.replace(W.srhd_double_tube(n), limiter=limiter, rk=rk)
        o = Oracle(w)
        run_to(o, t_end)
        U = o.state()
        P = o.cons_to_prim(np.moveaxis(U, 1, -1).reshape(-1, 5)).reshape(U.shape[0], *U.shape[2:], 5)
        rho = line_profile(w, np.moveaxis(P, -1, 1))
        x = (np.arange(n) + 0.5) / n
        ex = np.empty(n)
        r = x >= 0.5
        ex[r] = X.sample(inside, outside, g, (x[r] - 0.75) / t_end)[0]
        ex[~r] = X.sample(outside, inside, g, (x[~r] - 0.25) / t_end)[0]
        errs.append(np.abs(rho - ex).mean())
        assert np.ptp(U[:, 0], axis=(1, 2)).max() == 0.0     # uniform across the tube
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[0] > 0.45 and rates[1] > 0.75 and errs[-1] < 0.1, (errs, rates)
    ps, _ = X.star_state(inside, outside, g)
    v_s, rho_s, Vs = X.shock(outside, ps, g, +1)
    xs = 0.75 + Vs * t_end
    # the shock front: the last cell of the right half above the mid density
    # of the shell and the gas ahead of it
    right = (x > 0.75) & (rho > 0.5 * (rho_s + 1.0))
    cross = x[right].max() + 0.5 / n
    assert abs(cross - xs) < 3.0 / n, (cross, xs)
