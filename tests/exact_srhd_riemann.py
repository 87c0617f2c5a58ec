"""Exact solution of the 1-D Riemann problem of special relativistic
hydrodynamics (c = 1) for an ideal gas, h = 1 + g/(g-1) p/rho, without
tangential velocity.

Method of Marti & Mueller (J. Fluid Mech. 258, 317, 1994): the star pressure
p* is the root of v*_L(p) = v*_R(p).  Each side's star velocity follows, for
p above that side's pressure, from the Taub adiabat and the shock jump
conditions, and below it from the isentropic rarefaction, along which the
Riemann invariant artanh(v) +/- G(c_s) is constant, with
G(c_s) = 2/sqrt(g-1) artanh(c_s/sqrt(g-1)) the closed form of the integral of
c_s drho/rho for the ideal gas.  The self-similar solution is then sampled at
xi = x / t.  Used only to pin the oracle; independent of every other file in
the repo (the tests check it against the jump conditions and the Newtonian
limit).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def enthalpy(rho, p, g):
    return 1.0 + g / (g - 1.0) * p / rho


def sound_speed(rho, p, g):
    return math.sqrt(g * p / (rho * enthalpy(rho, p, g)))


def _G(cs, g):
    k = math.sqrt(g - 1.0)
    return 2.0 / k * math.atanh(cs / k)


def rarefaction(a, p, g, s):
    """State behind an isentropic rarefaction from a = (rho, v, p) down to
    pressure p; s = -1 for the left-facing wave, +1 for the right-facing one.
    Returns (v, rho)."""
    rho_a, v_a, p_a = a
    rho = rho_a * (p / p_a) ** (1.0 / g)
    J = math.atanh(v_a) - s * _G(sound_speed(rho_a, p_a, g), g)
    return math.tanh(J + s * _G(sound_speed(rho, p, g), g)), rho


def shock(a, p, g, s):
    """State behind a shock from a = (rho, v, p) up to pressure p; s = -1 for
    the left-facing shock, +1 for the right-facing one.  Returns
    (v, rho, shock speed)."""
    rho_a, v_a, p_a = a
    h_a = enthalpy(rho_a, p_a, g)
    dp = p - p_a
    # Taub adiabat [h^2] = (h_b/rho_b + h_a/rho_a)[p] with rho_b from the EOS:
    # a quadratic in h_b
    A = 1.0 - (g - 1.0) * dp / (g * p)
    B = (g - 1.0) * dp / (g * p)
    C = -h_a * h_a - h_a * dp / rho_a
    h_b = (-B + math.sqrt(B * B - 4.0 * A * C)) / (2.0 * A)
    rho_b = g * p / ((g - 1.0) * (h_b - 1.0))
    j2 = -dp / (h_b / rho_b - h_a / rho_a)          # squared mass flux through the shock
    j = s * math.sqrt(j2)
    W_a = 1.0 / math.sqrt(1.0 - v_a * v_a)
    D2 = (rho_a * W_a) ** 2
    Vs = (D2 * v_a + s * math.sqrt(j2) * math.sqrt(j2 + rho_a * rho_a)) / (D2 + j2)
    W_s = 1.0 / math.sqrt(1.0 - Vs * Vs)
    v_b = (h_a * W_a * v_a + W_s * dp / j) / (h_a * W_a + dp * (W_s * v_a / j + 1.0 / (rho_a * W_a)))
    return v_b, rho_b, Vs


def _side(a, p, g, s):
    if p > a[2]:
        v, rho, _ = shock(a, p, g, s)
    else:
        v, rho = rarefaction(a, p, g, s)
    return v, rho


def star_state(left, right, g):
    """(p*, v*) for left / right states (rho, v, p)."""
    f = lambda p: _side(left, p, g, -1)[0] - _side(right, p, g, +1)[0]
    lo = 1e-12 * min(left[2], right[2])
    hi = 1e3 * max(left[2], right[2])
    p = brentq(f, lo, hi, xtol=1e-300, rtol=1e-15, maxiter=500)
    return p, _side(left, p, g, -1)[0]


def sample(left, right, g, xi):
    """(rho, v, p) arrays of the exact solution at self-similar xi = x / t."""
    ps, vs = star_state(left, right, g)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    out = np.zeros((3, xi.size))
    for n, x in enumerate(xi):
        if x < vs:
            a, s = left, -1
        else:
            a, s = right, +1
        rho_a, v_a, p_a = a
        if ps > p_a:
            _, rho_s, Vs = shock(a, ps, g, s)
            behind = (x > Vs) if s < 0 else (x < Vs)
            out[:, n] = (rho_s, vs, ps) if behind else a
            continue
        _, rho_s = rarefaction(a, ps, g, s)
        c_a, c_s = sound_speed(rho_a, p_a, g), sound_speed(rho_s, ps, g)
        head = (v_a + s * c_a) / (1.0 + s * v_a * c_a)
        tail = (vs + s * c_s) / (1.0 + s * vs * c_s)
        if (s < 0 and x <= head) or (s > 0 and x >= head):
            out[:, n] = a
        elif (s < 0 and x >= tail) or (s > 0 and x <= tail):
            out[:, n] = (rho_s, vs, ps)
        else:
            def chi(p):
                v, rho = rarefaction(a, p, g, s)
                c = sound_speed(rho, p, g)
                return (v + s * c) / (1.0 + s * v * c) - x
            p = brentq(chi, ps, p_a, xtol=1e-300, rtol=1e-15, maxiter=500)
            v, rho = rarefaction(a, p, g, s)
            out[:, n] = (rho, v, p)
    return out
