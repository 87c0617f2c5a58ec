"""Exact solution of the 1-D Riemann problem for the ideal-gas Euler equations.

Textbook method (Toro 2009, Riemann Solvers and Numerical Methods for Fluid
Dynamics, ch. 4): Newton iteration for the star pressure on the pressure
functions f_L(p) + f_R(p) + (u_R - u_L) = 0, star velocity from the same
functions, then sampling of the self-similar solution at s = x / t.
Used only to pin the oracle; independent of every other file in the repo.
"""
from __future__ import annotations

import math

import numpy as np


def _f(p, rho, pk, g):
    a = math.sqrt(g * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    r = (p / pk) ** ((g - 1.0) / (2.0 * g))
    return 2.0 * a / (g - 1.0) * (r - 1.0), 1.0 / (rho * a) * (p / pk) ** (-(g + 1.0) / (2.0 * g))


def star_state(left, right, g):
    """(p*, u*) for left/right primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    al, ar = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    # two-rarefaction initial guess (Toro 4.46)
    z = (g - 1.0) / (2.0 * g)
    p = ((al + ar - 0.5 * (g - 1.0) * (ur - ul)) / (al / pl ** z + ar / pr ** z)) ** (1.0 / z)
    for _ in range(100):
        fl, dfl = _f(p, rl, pl, g)
        fr, dfr = _f(p, rr, pr, g)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(pn, 1e-14)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, g)
    fr, _ = _f(p, rr, pr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, g, s):
    """Exact (rho, u, p) at similarity coordinates s = x/t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, g)
    al, ar = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    s = np.asarray(s, dtype=np.float64)
    rho = np.empty_like(s)
    u = np.empty_like(s)
    p = np.empty_like(s)
    gm = (g - 1.0) / (g + 1.0)
    for q, x in np.ndenumerate(s):
        if x <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - al * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
                if x <= sl:
                    r, v, pp = rl, ul, pl
                else:
                    r = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
                    v, pp = us, ps
            else:  # left rarefaction
                shl = ul - al
                asl = al * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                stl = us - asl
                if x <= shl:
                    r, v, pp = rl, ul, pl
                elif x >= stl:
                    r = rl * (ps / pl) ** (1.0 / g)
                    v, pp = us, ps
                else:
                    c = 2.0 / (g + 1.0) + gm / al * (ul - x)
                    r = rl * c ** (2.0 / (g - 1.0))
                    v = 2.0 / (g + 1.0) * (al + 0.5 * (g - 1.0) * ul + x)
                    pp = pl * c ** (2.0 * g / (g - 1.0))
        else:
            if ps > pr:  # right shock
                sr = ur + ar * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
                if x >= sr:
                    r, v, pp = rr, ur, pr
                else:
                    r = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
                    v, pp = us, ps
            else:
                shr = ur + ar
                asr = ar * (ps / pr) ** ((g - 1.0) / (2.0 * g))
                str_ = us + asr
                if x >= shr:
                    r, v, pp = rr, ur, pr
                elif x <= str_:
                    r = rr * (ps / pr) ** (1.0 / g)
                    v, pp = us, ps
                else:
                    c = 2.0 / (g + 1.0) - gm / ar * (ur - x)
                    r = rr * c ** (2.0 / (g - 1.0))
                    v = 2.0 / (g + 1.0) * (-ar + 0.5 * (g - 1.0) * ur + x)
                    pp = pr * c ** (2.0 * g / (g - 1.0))
        rho[q], u[q], p[q] = r, v, pp
    return rho, u, p


def shock_speed(left, right, g):
    """Speed of the right-moving shock (assumes p* > p_R)."""
    rr, ur, pr = right
    ps, _ = star_state(left, right, g)
    ar = math.sqrt(g * pr / rr)
    return ur + ar * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))


def double_sod_density(x, t, g=1.4, hi=(1.0, 0.0, 1.0), lo=(0.125, 0.0, 0.1)):
    """Density of the periodic double Sod problem (high state in [1/4, 3/4])
    while the two wave fans have not met: for x >= 1/2 the Riemann problem at
    3/4 (high | low), for x < 1/2 its mirror image about x = 1/2."""
    x = np.asarray(x, dtype=np.float64)
    rho = np.empty_like(x)
    right = x >= 0.5
    r, _, _ = sample(hi, lo, g, (x[right] - 0.75) / t)
    rho[right] = r
    xm = 1.0 - x[~right]
    r, _, _ = sample(hi, lo, g, (xm - 0.75) / t)
    rho[~right] = r
    return rho
