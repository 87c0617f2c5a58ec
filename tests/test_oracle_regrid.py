"""Pins of the oracle's regrid pieces -- the Loehner estimator, the regrid
decision with 2:1 balance and the data transfer by point location -- against
closed forms, invariants and brute force.  CPU only."""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import pytest

from oracle import regrid as RG
from oracle.oracle import Oracle
from paper_2607_19277_amd import workloads as W

EPS = 0.01


def _with_rho(blocks, base, max_level, rho_of_index):
    """Euler state at rest, p = 1, density from the cell's global index on
    its level (i, j, k); the domain is base blocks wide (cubic cells)."""
    lo, hi = (0, 0, 0), tuple(float(b) for b in base)
    def prim(x, y, z, g, lev):
        n = [base[d] * 16 * 2.0 ** (lev - 1) for d in range(3)]
        i = np.rint((x - lo[0]) / (hi[0] - lo[0]) * n[0] - 0.5)
        j = np.rint((y - lo[1]) / (hi[1] - lo[1]) * n[1] - 0.5)
        k = np.rint((z - lo[2]) / (hi[2] - lo[2]) * n[2] - 0.5)
        rho = rho_of_index(i, j, k)
        zero = np.zeros_like(rho)
        return rho, zero, zero, zero, np.ones_like(rho)
    return W._make("regrid_test", W.EULER, W.HLLC, 1.4, 0.4, blocks, (16, 16, 16), base, lo, hi, max_level, prim)


# ---------------------------------------------------------------------------
# estimator

def test_lohner_zero_for_a_linear_field_away_from_the_seam():
    """Integer density 100 + i along x: every second difference is exactly
    zero except across the periodic seam, so the two inner blocks read 0."""
    w = _with_rho(W.uniform_blocks((4, 1, 1)), (4, 1, 1), 1, lambda i, j, k: 100.0 + i)
    e = Oracle(w).lohner(0, EPS)
    assert e[1] == 0.0 and e[2] == 0.0
    assert e[0] > 0.5 and e[3] > 0.5          # the seam jumps from 163 to 100


def test_lohner_closed_form_for_a_parabola():
    """rho = 1000 + (i - 32)^2 along x: a_x = 2, a_y = a_z = 0; the block value
    is the largest closed-form E over its cells."""
    w = _with_rho(W.uniform_blocks((4, 1, 1)), (4, 1, 1), 1, lambda i, j, k: 1000.0 + (i - 32.0) ** 2)
    e = Oracle(w).lohner(0, EPS)
    for q in (1, 2):
        i = np.arange(16 * q, 16 * q + 16, dtype=float)
        r = 1000.0 + (i - 32.0) ** 2
        rp, rm = 1000.0 + (i - 31.0) ** 2, 1000.0 + (i - 33.0) ** 2
        bx = (np.abs(rp - r) + np.abs(r - rm)) + EPS * ((np.abs(rp) + 2 * np.abs(r)) + np.abs(rm))
        bt = EPS * 4 * r                       # y and z: constant neighbours
        ref = np.sqrt(4.0 / ((bx * bx + bt * bt) + bt * bt)).max()
        assert abs(e[q] - ref) <= 1e-15 * ref, (q, e[q], ref)


def test_lohner_of_a_jump_and_its_range():
    """A density jump from 1 to 2 at x = 1/2: the cell next to it has
    a_x = 1, b_x = 1 + eps (1 + 2 + 2)... E close to 1; E stays in [0, 1]
    everywhere (|a| <= b) on a random smooth AMR state as well."""
    w = _with_rho(W.uniform_blocks((4, 1, 1)), (4, 1, 1), 1, lambda i, j, k: np.where(i < 32, 1.0, 2.0))
    e = Oracle(w).lohner(0, EPS)
    # cell i = 31: u- = 1, u = 1, u+ = 2 -> a = 1, b_x = 1 + eps*5, b_y = b_z = eps*4
    ref = 1.0 / math.sqrt((1.0 + EPS * 5.0) ** 2 + 2 * (EPS * 4.0) ** 2)
    assert abs(e[1] - ref) <= 1e-15 and abs(e[2] - 1.0 / math.sqrt((1 + EPS * 7) ** 2 + 2 * (EPS * 8) ** 2)) <= 1e-15
    blocks = W.nested_blocks((4, 4, 4), 2)
    e2 = Oracle(W.smooth_random(blocks, (4, 4, 4), 2, seed=5)).lohner(0, EPS)
    assert np.all(e2 >= 0.0) and np.all(e2 <= 1.0) and e2.max() > 0.0


def test_lohner_zero_where_the_variable_vanishes():
    """Gas at rest: the momentum is exactly zero on every stencil, where both
    of the estimator's sums vanish; the estimate is then 0 (not 0/0).  With the
    momentum zero in the left half of the box and a jump to 1 in the right
    half, the left inner block reads 0, the blocks at the jumps read the
    closed form of a unit step and nothing is NaN."""
    w = _with_rho(W.uniform_blocks((4, 1, 1)), (4, 1, 1), 1, lambda i, j, k: 1.0 + 0.01 * i)
    o = Oracle(w)
    for v in (1, 2, 3):
        e = o.lohner(v, EPS)
        assert np.all(e == 0.0), (v, e)
    U = w.U.copy()
    for b in range(4):
        U[b, 1] = 0.0 if b < 2 else 1.0
    e = Oracle(dataclasses.replace(w, U=U)).lohner(1, EPS)
    assert not np.any(np.isnan(e))
    assert e[0] > 0.5 and e[1] > 0.5 and e[2] > 0.5 and e[3] > 0.5    # seam at x = 0 and jump at x = 1/2
    w2 = _with_rho(W.uniform_blocks((8, 1, 1)), (8, 1, 1), 1, lambda i, j, k: 1.0 + 0.0 * i)
    U2 = w2.U.copy()
    U2[4:, 1] = 1.0
    e2 = Oracle(dataclasses.replace(w2, U=U2)).lohner(1, EPS)
    assert e2[1] == 0.0 and e2[2] == 0.0                               # zero on every stencil
    ref = 1.0 / math.sqrt((1.0 + EPS * 1.0) ** 2 + 2 * (EPS * 0.0) ** 2)  # u- = u = 0, u+ = 1
    assert abs(e2[3] - ref) <= 1e-15, (e2[3], ref)


# ---------------------------------------------------------------------------
# decision

def _dense_levels(leaves, base, L):
    """Level of the covering leaf for every level-L block (brute force);
    asserts that the leaves tile the domain exactly once."""
    n = [b << (L - 1) for b in base]
    lev = np.zeros(n[::-1], dtype=int)
    for (l, x, y, z) in leaves:
        s = 1 << (L - l)
        sl = lev[z * s:(z + 1) * s, y * s:(y + 1) * s, x * s:(x + 1) * s]
        assert np.all(sl == 0), "overlap"
        sl[...] = l
    assert np.all(lev > 0), "gap"
    return lev


def _check_balanced(leaves, base, L):
    lev = _dense_levels(leaves, base, L)
    for ax in range(3):
        d = np.abs(lev - np.roll(lev, 1, axis=ax))
        assert d.max() <= 1, "2:1 violated"


def test_decide_no_change_and_single_refinement():
    b = W.uniform_blocks((2, 2, 2))
    new, R, P = RG.decide(b, np.zeros(8), (2, 2, 2), 3, 0.5, 0.1)
    assert new == sorted(tuple(r) for r in b.tolist()) and R == [] and P == []
    err = np.zeros(8)
    err[3] = 0.9
    new, R, P = RG.decide(b, err, (2, 2, 2), 3, 0.5, -1.0)
    assert R == [tuple(b[3])] and len(new) == 15
    _check_balanced(new, (2, 2, 2), 2)


def test_decide_refinement_propagates_for_balance():
    """Refining a level-2 leaf next to a level-1 leaf refines that leaf too."""
    base = (4, 4, 4)
    b = W.refine_blocks(W.uniform_blocks(base), [0])            # children of block (0,0,0)
    leaves = [tuple(r) for r in b.tolist()]
    q = leaves.index((2, 1, 0, 0))                               # touches level-1 block (1,0,0)
    err = np.zeros(len(leaves))
    err[q] = 0.9
    new, R, P = RG.decide(b, err, base, 3, 0.5, -1.0)
    assert (2, 1, 0, 0) in R and (1, 1, 0, 0) in R
    _check_balanced(new, base, 3)


def test_decide_coarsening_and_its_balance_veto():
    base = (4, 4, 4)
    b = W.refine_blocks(W.uniform_blocks(base), [0])
    leaves = [tuple(r) for r in b.tolist()]
    new, R, P = RG.decide(b, np.zeros(len(leaves)), base, 3, 0.5, 0.1)
    assert P == [(1, 0, 0, 0)] and new == sorted(tuple(r) for r in W.uniform_blocks(base).tolist())
    # one child above the coarsening threshold keeps the octet
    err = np.zeros(len(leaves))
    err[leaves.index((2, 1, 1, 0))] = 0.3
    new, R, P = RG.decide(b, err, base, 3, 0.5, 0.1)
    assert P == [] and R == [] and new == sorted(leaves)
    # a level-3 region next to the octet forbids coarsening it back to level 1
    u = W.uniform_blocks(base)
    ul = [tuple(r) for r in u.tolist()]
    e1 = np.array([0.9 if r in ((1, 0, 0, 0), (1, 1, 0, 0)) else 0.0 for r in ul])
    m2 = np.array(RG.decide(u, e1, base, 3, 0.5, -1.0)[0], dtype=np.int32)
    l2 = [tuple(r) for r in m2.tolist()]
    e2 = np.array([0.9 if r == (2, 2, 0, 0) else 0.0 for r in l2])
    m3 = np.array(RG.decide(m2, e2, base, 3, 0.5, -1.0)[0], dtype=np.int32)
    l3 = [tuple(r) for r in m3.tolist()]
    _check_balanced(l3, base, 3)
    octet = [(2, x, y, z) for z in (0, 1) for y in (0, 1) for x in (0, 1)]
    assert all(k in l3 for k in octet) and (3, 4, 0, 0) in l3
    e3 = np.array([0.0 if r in octet else 1.0 for r in l3])
    new, R, P = RG.decide(m3, e3, base, 3, 2.0, 0.5)
    assert P == [] and R == [] and new == sorted(l3)


@pytest.mark.parametrize("seed", range(6))
def test_decide_random_meshes_stay_balanced(seed):
    rng = np.random.default_rng(seed)
    base = (3, 3, 2)
    blocks = W.uniform_blocks(base)
    for _ in range(2):                                          # a random balanced 3-level mesh
        err = rng.random(len(blocks))
        new, _, _ = RG.decide(blocks, err, base, 3, 0.7, -1.0)
        blocks = np.array(new, dtype=np.int32)
    err = rng.random(len(blocks))
    new, R, P = RG.decide(blocks, err, base, 3, 0.6, 0.3)
    _check_balanced(new, base, 3)
    for (b, e) in zip([tuple(r) for r in blocks.tolist()], err):
        if e > 0.6 and b[0] < 3:
            assert b not in new, "flagged leaf not refined"


# ---------------------------------------------------------------------------
# data transfer

def test_remap_identity_and_conservation():
    base = (2, 2, 2)
    w = W.smooth_random(W.nested_blocks((4, 4, 4), 2), (4, 4, 4), 2, seed=3)
    o = Oracle(w)
    same = o.remap(w.blocks)
    assert np.array_equal(same, w.U)
    leaves = [tuple(r) for r in w.blocks.tolist()]
    err = np.zeros(len(leaves))
    err[:5] = 0.9
    new, R, P = RG.decide(w.blocks, err, w.base, 3, 0.5, 0.05)
    assert R and P
    U2 = o.remap(new)
    vol_old = np.array([w.dx(b[0]) ** 3 for b in leaves])
    vol_new = np.array([w.dx(b[0]) ** 3 for b in new])
    for v in range(5):
        a = math.fsum((w.U[:, v] * vol_old[:, None, None, None]).ravel())
        c = math.fsum((U2[:, v] * vol_new[:, None, None, None]).ravel())
        assert abs(a - c) <= 1e-13 * max(1.0, abs(a)), (v, a, c)


def test_remap_prolongation_is_exact_for_linear_fields_and_restriction_inverts_it():
    """Density 2 + i/4 along x (dyadic, so every operation is exact): the
    children of a refined block hold the same linear field at their centres,
    and restricting them gives the parent back."""
    base = (4, 1, 1)
    w = _with_rho(W.uniform_blocks(base), base, 2, lambda i, j, k: 2.0 + i / 4.0)
    o = Oracle(w)
    new = sorted(tuple(r) for r in W.refine_blocks(w.blocks, [1]).tolist())
    U2 = o.remap(new)
    for q, (l, x, y, z) in enumerate(new):
        if l == 2:
            i = np.arange(16 * x, 16 * x + 16)
            ref = 2.0 + (i / 2.0 - 0.25) / 4.0            # fine centre i -> coarse coordinate (i - 1/2)/2
            assert np.array_equal(U2[q, 0], np.broadcast_to(ref, (16, 16, 16)))
    w2 = dataclasses.replace(w, blocks=np.array(new, dtype=np.int32), U=U2)
    back = Oracle(w2).remap(w.blocks)
    assert np.array_equal(back, w.U)
