"""Seeded synthetic inputs: block meshes and initial conserved states.

This module is shared by the HIP path's tests/benchmark and by the CPU oracle.
It holds none of the update's arithmetic: it only lays out block lists and
samples initial conditions at cell centres.  Turning an initial primitive
state into conserved variables uses the ideal-gas closure of the hydro and
MHD modules (Sec. 2.3.1 closure; Sec. 2.3.3 total energy), which is part of
stating the initial condition, not of the solver.

Random numbers: SplitMix64 (Steele, Lea & Flood 2014) keyed by
(seed, global cell index on its level, component); a uniform double is the
top 53 bits times 2^-53.  The draw therefore does not depend on how the
domain is cut into blocks.

Array conventions (shared by the C-ABI and the oracle):
  blocks : int32 [n, 4] rows (level, ix, iy, iz), block coordinates on that
           level, level 1 = base grid;
  U      : float64 [n, nvar, bz, by, bx] interior cells, x fastest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

EULER, MHD, SRHD = 0, 1, 2
HLL, HLLC, LF = 0, 1, 2
MINMOD, VANLEER = 0, 1
FP64, FP32_FLUX = 0, 1

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to x + golden gamma (uint64, wrapping)."""
    with np.errstate(over="ignore"):
        z = (np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, index: np.ndarray, comp: int) -> np.ndarray:
    """Uniform [0,1) doubles for (seed, cell index, component)."""
    key = splitmix64(np.uint64(seed))
    with np.errstate(over="ignore"):
        x = key + np.asarray(index, dtype=np.uint64) * np.uint64(8) + np.uint64(comp)
    return (splitmix64(x) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform(seed: int, index: np.ndarray, comp: int, lo: float, hi: float) -> np.ndarray:
    return lo + (hi - lo) * uniform01(seed, index, comp)


@dataclass
class Workload:
    """A mesh, its initial conserved state and the solver parameters."""
    name: str
    physics: int
    riemann: int
    gamma: float
    cfl: float
    bn: tuple
    base: tuple
    lo: tuple
    hi: tuple
    max_level: int
    blocks: np.ndarray
    U: np.ndarray
    steps: int = 1
    glm_alpha: float = 0.5
    extra: dict = field(default_factory=dict)
    limiter: int = 0          # reconstruction slope: 0 minmod, 1 van Leer
    rk: int = 2               # SSP Runge-Kutta stages: 2 or 3

    @property
    def nvar(self) -> int:
        return 9 if self.physics == MHD else 5

    @property
    def nblocks(self) -> int:
        return int(self.blocks.shape[0])

    @property
    def ncells(self) -> int:
        return int(self.nblocks * self.bn[0] * self.bn[1] * self.bn[2])

    def dx(self, level: int = 1) -> float:
        return (self.hi[0] - self.lo[0]) / (self.base[0] * self.bn[0]) / 2 ** (level - 1)


# ---------------------------------------------------------------------------
# meshes

def uniform_blocks(base) -> np.ndarray:
    """All level-1 blocks, z slowest, x fastest."""
    bx, by, bz = base
    iz, iy, ix = np.meshgrid(np.arange(bz), np.arange(by), np.arange(bx), indexing="ij")
    n = bx * by * bz
    out = np.empty((n, 4), dtype=np.int32)
    out[:, 0] = 1
    out[:, 1] = ix.ravel()
    out[:, 2] = iy.ravel()
    out[:, 3] = iz.ravel()
    return out


def nested_blocks(base, nlevels: int, frac=(0.25, 0.75)) -> np.ndarray:
    """Static nested refinement: level l+1 covers the central half (per axis)
    of the level-l refined region; returns the leaves, coarsest level first."""
    regions = []          # per level: (lo, hi) block-index box on that level
    lo = np.zeros(3, dtype=np.int64)
    hi = np.array(base, dtype=np.int64)
    regions.append((lo, hi))
    for l in range(2, nlevels + 1):
        plo, phi = regions[-1]
        ext = phi - plo
        if np.any(ext % 4):
            raise ValueError("refined box must split into whole blocks")
        clo = plo + ext // 4
        chi = phi - ext // 4
        regions.append((2 * clo, 2 * chi))
    rows = []
    for l in range(1, nlevels + 1):
        lo_, hi_ = regions[l - 1]
        for iz in range(lo_[2], hi_[2]):
            for iy in range(lo_[1], hi_[1]):
                for ix in range(lo_[0], hi_[0]):
                    if l < nlevels:
                        clo, chi = regions[l]
                        c = np.array([2 * ix, 2 * iy, 2 * iz])
                        if np.all(c >= clo) and np.all(c < chi):
                            continue
                    rows.append((l, ix, iy, iz))
    return np.array(rows, dtype=np.int32)


def refine_blocks(blocks: np.ndarray, which) -> np.ndarray:
    """Replace the listed blocks (indices) by their 8 children."""
    which = set(int(q) for q in which)
    rows = []
    for q, (l, ix, iy, iz) in enumerate(blocks.tolist()):
        if q in which:
            for dz in (0, 1):
                for dy in (0, 1):
                    for dx in (0, 1):
                        rows.append((l + 1, 2 * ix + dx, 2 * iy + dy, 2 * iz + dz))
        else:
            rows.append((l, ix, iy, iz))
    return np.array(rows, dtype=np.int32)


def cell_coords(blocks: np.ndarray, bn, base, lo, hi):
    """Cell-centre coordinates and global cell indices per level.
    Returns x, y, z (float64) and gidx (int64), each [n, bz, by, bx]."""
    blocks = np.asarray(blocks)
    n = blocks.shape[0]
    bx, by, bz = bn
    dx1 = (hi[0] - lo[0]) / (base[0] * bx)
    lev = blocks[:, 0].astype(np.int64)
    dx = dx1 / (2.0 ** (lev - 1))
    ii = np.arange(bx)[None, None, None, :]
    jj = np.arange(by)[None, None, :, None]
    kk = np.arange(bz)[None, :, None, None]
    gi = blocks[:, 1].astype(np.int64)[:, None, None, None] * bx + ii
    gj = blocks[:, 2].astype(np.int64)[:, None, None, None] * by + jj
    gk = blocks[:, 3].astype(np.int64)[:, None, None, None] * bz + kk
    d4 = dx[:, None, None, None]
    x = lo[0] + (gi + 0.5) * d4
    y = lo[1] + (gj + 0.5) * d4
    z = lo[2] + (gk + 0.5) * d4
    nx = (base[0] * bx) * (2 ** (lev - 1))
    ny = (base[1] * by) * (2 ** (lev - 1))
    gidx = (gk * ny[:, None, None, None] + gj) * nx[:, None, None, None] + gi
    shape = (n, bz, by, bx)
    return (np.broadcast_to(x, shape), np.broadcast_to(y, shape),
            np.broadcast_to(z, shape), np.broadcast_to(gidx, shape))


def srhd_prim_to_cons(gamma, rho, vx, vy, vz, p) -> np.ndarray:
    """Initial SRHD state (D, m, tau) from rho, the 3-velocity (|v| < 1) and p
    with the ideal-gas enthalpy h = 1 + gamma/(gamma-1) p/rho."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = np.broadcast_shapes(rho.shape, np.shape(vx), np.shape(vy), np.shape(vz), np.shape(p))
    rho, vx, vy, vz, p = (np.broadcast_to(np.asarray(a, dtype=np.float64), shape) for a in (rho, vx, vy, vz, p))
    G = 1.0 / np.sqrt(1.0 - ((vx * vx + vy * vy) + vz * vz))
    rhoh = rho + gamma / (gamma - 1.0) * p
    U = np.empty((shape[0], 5) + shape[1:], dtype=np.float64)
    U[:, 0] = G * rho
    U[:, 1] = G * G * rhoh * vx
    U[:, 2] = G * G * rhoh * vy
    U[:, 3] = G * G * rhoh * vz
    U[:, 4] = G * G * rhoh - p - G * rho
    return U


def prim_to_cons(gamma, rho, vx, vy, vz, p, B=None, psi=None) -> np.ndarray:
    """Initial conserved state from primitives (ideal-gas closure)."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = np.broadcast_shapes(rho.shape, np.shape(vx), np.shape(vy), np.shape(vz), np.shape(p))
    nvar = 5 if B is None else 9
    U = np.empty((shape[0], nvar) + shape[1:], dtype=np.float64)
    rho = np.broadcast_to(rho, shape)
    vx, vy, vz, p = (np.broadcast_to(np.asarray(a, dtype=np.float64), shape) for a in (vx, vy, vz, p))
    U[:, 0] = rho
    U[:, 1] = rho * vx
    U[:, 2] = rho * vy
    U[:, 3] = rho * vz
    e = p / (gamma - 1.0) + 0.5 * rho * ((vx * vx + vy * vy) + vz * vz)
    if B is not None:
        bx_, by_, bz_ = (np.broadcast_to(np.asarray(b, dtype=np.float64), shape) for b in B)
        e = e + 0.5 * ((bx_ * bx_ + by_ * by_) + bz_ * bz_)
        U[:, 5] = bx_
        U[:, 6] = by_
        U[:, 7] = bz_
        U[:, 8] = 0.0 if psi is None else np.broadcast_to(psi, shape)
    U[:, 4] = e
    return U


def _make(name, physics, riemann, gamma, cfl, blocks, bn, base, lo, hi, max_level, prim_fn, steps=1, **extra):
    """prim_fn returns (rho, vx, vy, vz, p) for Euler or, for MHD,
    (rho, vx, vy, vz, p, Bx, By, Bz, psi)."""
    x, y, z, gidx = cell_coords(blocks, bn, base, lo, hi)
    lev = np.broadcast_to(np.asarray(blocks)[:, 0].astype(np.int64)[:, None, None, None], x.shape)
    prims = prim_fn(x, y, z, gidx, lev)
    if physics == MHD:
        U = prim_to_cons(gamma, *prims[:5], B=prims[5:8], psi=prims[8])
    elif physics == SRHD:
        U = srhd_prim_to_cons(gamma, *prims)
    else:
        U = prim_to_cons(gamma, *prims)
    return Workload(name, physics, riemann, gamma, cfl, tuple(bn), tuple(base), tuple(lo), tuple(hi),
                    max_level, np.asarray(blocks, dtype=np.int32), np.ascontiguousarray(U), steps, extra=extra)


# ---------------------------------------------------------------------------
# the five benchmark configurations and the test problems

def uniform_random(nb=4, seed=1, riemann=HLL, steps=10) -> Workload:
    """Uniform periodic box of nb^3 blocks of 16^3 cells: rho = 1 + 0.1 sin(2 pi x),
    p = 1, each velocity component of each cell uniform in [-0.1, 0.1].
    nb = 4 gives the 64^3 ten-step parity configuration (HLL, CFL 0.4)."""
    def prim(x, y, z, g, lev):
        rho = 1.0 + 0.1 * np.sin(2.0 * np.pi * x)
        return (rho, uniform(seed, g, 0, -0.1, 0.1), uniform(seed, g, 1, -0.1, 0.1),
                uniform(seed, g, 2, -0.1, 0.1), np.ones_like(rho))
    base = (nb, nb, nb)
    return _make(f"uniform{16 * nb}", EULER, riemann, 5.0 / 3.0, 0.4, uniform_blocks(base), (16, 16, 16),
                 base, (0, 0, 0), (1, 1, 1), 1, prim, steps=steps)


def sedov(base_blocks=8, nlevels=4, riemann=HLLC, p_amb=1e-5, energy=1.0, steps=20) -> Workload:
    """Point blast on static nested levels: base (16*base_blocks)^3, each finer level
    covering the central half of its parent, energy deposited in the central 2^3
    finest cells.  base_blocks=8, nlevels=4 gives 1856 leaves (448+448+448+512)."""
    gamma = 5.0 / 3.0
    blocks = nested_blocks((base_blocks,) * 3, nlevels)
    nfine = 16 * base_blocks * 2 ** (nlevels - 1)
    dxf = 1.0 / nfine
    half = nfine // 2

    def prim(x, y, z, g, lev):
        rho = np.ones(x.shape)
        p = np.full(x.shape, p_amb)
        # energy density added to the 8 finest cells around the centre; as a
        # pressure increment dp = (gamma-1) de
        gi = np.floor(x / dxf).astype(np.int64)
        gj = np.floor(y / dxf).astype(np.int64)
        gk = np.floor(z / dxf).astype(np.int64)
        fine = (lev == nlevels)
        hit = fine & (gi >= half - 1) & (gi <= half) & (gj >= half - 1) & (gj <= half) & (gk >= half - 1) & (gk <= half)
        p = np.where(hit, p + (gamma - 1.0) * (energy / 8.0) / dxf ** 3, p)
        return rho, 0.0, 0.0, 0.0, p
    w = _make(f"sedov{16 * base_blocks}_L{nlevels}", EULER, riemann, gamma, 0.4, blocks, (16, 16, 16),
              (base_blocks,) * 3, (0, 0, 0), (1, 1, 1), nlevels, prim, steps=steps)
    return w


def kelvin_helmholtz(n=256, seed=3, riemann=HLLC, t_end=0.5, bn=16) -> Workload:
    """Shear layer: rho = 2, v_x = +0.5 inside |y - 0.5| < 0.25, else rho = 1,
    v_x = -0.5; v_y = 0.01 sin(4 pi x) + U[-1e-3, 1e-3]; v_z = U[-1e-3, 1e-3]; p = 2.5.
    bn: cells per block edge (the random draws follow the global cell index, so
    every block size gives the same cell values)."""
    def prim(x, y, z, g, lev):
        inside = np.abs(y - 0.5) < 0.25
        rho = np.where(inside, 2.0, 1.0)
        vx = np.where(inside, 0.5, -0.5)
        vy = 0.01 * np.sin(4.0 * np.pi * x) + uniform(seed, g, 1, -1e-3, 1e-3)
        vz = uniform(seed, g, 2, -1e-3, 1e-3)
        return rho, vx, vy, vz, np.full(x.shape, 2.5)
    nb = n // bn
    base = (nb, nb, nb)
    return _make(f"kh{n}" + ("" if bn == 16 else f"_b{bn}"), EULER, riemann, 5.0 / 3.0, 0.4, uniform_blocks(base),
                 (bn, bn, bn), base,
                 (0, 0, 0), (1, 1, 1), 1, prim, steps=1, t_end=t_end)


def double_sod(ncell=256, axis=0, bn_long=16, bn_short=2, riemann=HLLC, gamma=1.4) -> Workload:
    """Periodic double Sod tube along `axis`: (rho, p) = (1, 1) in [1/4, 3/4],
    (0.125, 0.1) outside, at rest; uniform across.  Blocks are bn_long cells
    along the axis and bn_short across (one block across)."""
    bn = [bn_short] * 3
    bn[axis] = bn_long
    base = [1, 1, 1]
    base[axis] = ncell // bn_long
    lo = (0.0, 0.0, 0.0)
    hi = [bn_short / ncell] * 3
    hi[axis] = 1.0

    def prim(x, y, z, g, lev):
        s = (x, y, z)[axis]
        inside = (s > 0.25) & (s < 0.75)
        rho = np.where(inside, 1.0, 0.125)
        p = np.where(inside, 1.0, 0.1)
        return rho, 0.0, 0.0, 0.0, p
    return _make(f"dsod{ncell}", EULER, riemann, gamma, 0.4, uniform_blocks(tuple(base)), tuple(bn),
                 tuple(base), lo, tuple(hi), 1, prim)


def density_wave(blocks, base, bn=(16, 16, 16), vel=(1.0, 0.5, 0.25), amp=0.2, riemann=HLLC,
                 gamma=5.0 / 3.0, max_level=1, kvec=(1, 1, 1)) -> Workload:
    """Smooth advected density wave rho = 1 + amp sin(2 pi k.x), uniform
    velocity and p = 1 (exact solution: translation)."""
    def prim(x, y, z, g, lev):
        rho = 1.0 + amp * np.sin(2.0 * np.pi * ((kvec[0] * x + kvec[1] * y) + kvec[2] * z))
        return rho, vel[0], vel[1], vel[2], np.ones(x.shape)
    return _make("dwave", EULER, riemann, gamma, 0.4, blocks, bn, base, (0, 0, 0),
                 tuple(b * n / (base[0] * bn[0]) for b, n in zip(base, bn)), max_level, prim)


def constant_state(blocks, base, max_level, rho=1.3, v=(0.2, -0.1, 0.3), p=0.7, riemann=HLLC, physics=EULER,
                   B=(0.3, -0.2, 0.1), gamma=5.0 / 3.0) -> Workload:
    def prim(x, y, z, g, lev):
        return rho * np.ones(x.shape), v[0], v[1], v[2], p * np.ones(x.shape)
    bn = (16, 16, 16)
    w = _make("const", EULER, riemann, gamma, 0.4, blocks, bn, base, (0, 0, 0), (1, 1, 1), max_level, prim)
    if physics == MHD:
        x, y, z, g = cell_coords(blocks, bn, base, (0, 0, 0), (1, 1, 1))
        w.U = prim_to_cons(gamma, rho * np.ones(x.shape), v[0], v[1], v[2], p * np.ones(x.shape), B=B, psi=0.0)
        w.physics = MHD
        w.riemann = HLL
    return w


def smooth_random(blocks, base, max_level, seed=7, riemann=HLLC, gamma=5.0 / 3.0, nmodes=4, bn=16) -> Workload:
    """Smooth positive state with a few seeded Fourier modes per field, on any
    mesh of blocks of bn^3 cells."""
    rng_amp = uniform(seed, np.arange(4 * nmodes * 5), 0, -1.0, 1.0)
    ks = (splitmix64(np.arange(3 * nmodes * 5, dtype=np.uint64) + np.uint64(seed)) % np.uint64(2)).astype(np.int64) + 1

    def field(x, y, z, f):
        s = np.zeros(x.shape)
        for q in range(nmodes):
            a = rng_amp[4 * (f * nmodes + q)]
            ph = np.pi * rng_amp[4 * (f * nmodes + q) + 1]
            k = ks[3 * (f * nmodes + q):3 * (f * nmodes + q) + 3]
            s = s + a * np.sin(2.0 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
        return s / nmodes

    def prim(x, y, z, g, lev):
        rho = 1.25 + 0.5 * field(x, y, z, 0)
        p = 1.25 + 0.5 * field(x, y, z, 1)
        return rho, 0.3 * field(x, y, z, 2), 0.3 * field(x, y, z, 3), 0.3 * field(x, y, z, 4), p
    return _make("smooth", EULER, riemann, gamma, 0.4, blocks, (bn, bn, bn), base, (0, 0, 0), (1, 1, 1),
                 max_level, prim)


def permute(w: Workload, seed: int = 11) -> Workload:
    """Same workload with its blocks listed in a seeded random order."""
    key = splitmix64(np.arange(w.nblocks, dtype=np.uint64) + np.uint64(seed))
    order = np.argsort(key, kind="stable")
    return Workload(w.name + "_perm", w.physics, w.riemann, w.gamma, w.cfl, w.bn, w.base, w.lo, w.hi,
                    w.max_level, np.ascontiguousarray(w.blocks[order]), np.ascontiguousarray(w.U[order]),
                    w.steps, w.glm_alpha, dict(w.extra, order=order))


# ---------------------------------------------------------------------------
# ideal MHD with GLM cleaning (nvar = 9: rho, m, e, B, psi)

def mhd_smooth_random(blocks, base, max_level, seed=9, b_amp=0.6, psi_amp=0.0, gamma=5.0 / 3.0) -> Workload:
    """Smooth positive MHD state on any mesh: the hydro fields of smooth_random
    plus a smooth magnetic field of amplitude ~b_amp (not divergence free) and
    optionally a smooth psi."""
    h = smooth_random(blocks, base, max_level, seed=seed, gamma=gamma)
    amp = uniform(seed + 1, np.arange(12), 0, -1.0, 1.0)

    def prim(x, y, z, g, lev):
        U = h.U
        rho = U[:, 0]
        vx, vy, vz = U[:, 1] / rho, U[:, 2] / rho, U[:, 3] / rho
        p = (gamma - 1.0) * (U[:, 4] - 0.5 * rho * ((vx * vx + vy * vy) + vz * vz))
        B = [b_amp * (0.5 + 0.5 * amp[3 * d]) * np.sin(2.0 * np.pi * ((x if d != 0 else y) + amp[3 * d + 1]))
             + b_amp * 0.5 * amp[3 * d + 2] * np.cos(2.0 * np.pi * (z if d != 2 else x)) for d in range(3)]
        psi = psi_amp * np.sin(2.0 * np.pi * (x + y + z))
        return rho, vx, vy, vz, p, B[0], B[1], B[2], psi
    return _make("mhd_smooth", MHD, HLL, gamma, 0.4, blocks, (16, 16, 16), base, (0, 0, 0), (1, 1, 1),
                 max_level, prim)


def mhd_constant(blocks, base, max_level, rho=1.2, v=(0.3, -0.2, 0.1), p=0.8, B=(0.7, 0.0, 0.0), psi=0.0,
                 gamma=5.0 / 3.0) -> Workload:
    def prim(x, y, z, g, lev):
        one = np.ones(x.shape)
        return rho * one, v[0], v[1], v[2], p * one, B[0] * one, B[1] * one, B[2] * one, psi * one
    return _make("mhd_const", MHD, HLL, gamma, 0.4, blocks, (16, 16, 16), base, (0, 0, 0), (1, 1, 1),
                 max_level, prim)


def alfven_wave(ncell=64, bn_long=16, bn_short=2, amp=0.1, b_par=1.0, p=0.1, gamma=5.0 / 3.0) -> Workload:
    """Circularly polarised Alfven wave along x (periodic, length 1): rho = 1,
    B = (b_par, amp sin 2 pi x, amp cos 2 pi x), v = -(0, B_y, B_z)/sqrt(rho),
    uniform p; an exact nonlinear solution travelling at b_par/sqrt(rho)
    (period 1 for b_par = 1).  Blocks are bn_long cells along x and bn_short
    across (one block across)."""
    bn = (bn_long, bn_short, bn_short)
    base = (ncell // bn_long, 1, 1)
    hi = (1.0, bn_short / ncell, bn_short / ncell)

    def prim(x, y, z, g, lev):
        by = amp * np.sin(2.0 * np.pi * x)
        bz = amp * np.cos(2.0 * np.pi * x)
        one = np.ones(x.shape)
        return one, 0.0 * one, -by, -bz, p * one, b_par * one, by, bz, 0.0 * one
    return _make(f"alfven{ncell}", MHD, HLL, gamma, 0.4, uniform_blocks(base), bn, base, (0, 0, 0), hi, 1, prim)


def _balance(leaves: set, base) -> set:
    """Refine leaves until no face neighbour (periodic) is two or more levels
    finer; leaves are (level, ix, iy, iz)."""
    def covering(l, i):
        """leaf containing level-l block i, or None if that region is finer."""
        for lv in range(l, 0, -1):
            sh = l - lv
            key = (lv, i[0] >> sh, i[1] >> sh, i[2] >> sh)
            if key in leaves:
                return key
        return None
    changed = True
    while changed:
        changed = False
        for (l, ix, iy, iz) in sorted(leaves, key=lambda t: -t[0]):
            n = [b << (l - 1) for b in base]
            for d in range(3):
                for s in (-1, 1):
                    j = [ix, iy, iz]
                    j[d] = (j[d] + s) % n[d]
                    c = covering(l, j)
                    if c is not None and c[0] < l - 1:       # coarser by two: refine it
                        leaves.discard(c)
                        cl, cx, cy, cz = c
                        for dz in (0, 1):
                            for dy in (0, 1):
                                for dx in (0, 1):
                                    leaves.add((cl + 1, 2 * cx + dx, 2 * cy + dy, 2 * cz + dz))
                        changed = True
                        break
                if changed:
                    break
            if changed:
                break
    return leaves


def orszag_tang_mesh(base=(8, 8, 2), nlevels=4, threshold=0.55, step=-0.1):
    """Static 2:1 mesh for the z-uniform Orszag-Tang vortex.  Reading: the
    initial density is uniform, so no density gradient exists to refine on at
    t = 0; blocks are refined where the initial current density
    |J_z| = |dB_y/dx - dB_x/dy| (the current sheets where the density fronts
    of the vortex form) is large: a level-l block is refined when the mean of
    |J_z| / max |J_z| over its cell centres is at least threshold + (l-1) step;
    then 2:1 balance is enforced.  The defaults give 18 944 leaves (77.6 M
    cells) on levels 2-4 of a four-level hierarchy over a 128 x 128 x 32 base
    grid (balance refines every base block)."""
    def indicator(l, ix, iy):
        dx = 1.0 / (base[0] * 16 * 2 ** (l - 1))
        x = (ix * 16 + np.arange(16) + 0.5) * dx
        y = (iy * 16 + np.arange(16) + 0.5) * dx
        # J_z sqrt(4 pi) = 4 pi cos(4 pi x) + 2 pi cos(2 pi y); max 6 pi
        j = np.abs(2.0 * np.cos(4 * np.pi * x)[None, :] + np.cos(2 * np.pi * y)[:, None]) / 3.0
        return float(j.mean())
    leaves = {(1, ix, iy, iz) for ix in range(base[0]) for iy in range(base[1]) for iz in range(base[2])}
    for l in range(1, nlevels):
        cut = threshold + (l - 1) * step
        for (lv, ix, iy, iz) in [b for b in leaves if b[0] == l]:
            if indicator(l, ix, iy) >= cut:
                leaves.discard((lv, ix, iy, iz))
                for dz in (0, 1):
                    for dy in (0, 1):
                        for dx in (0, 1):
                            leaves.add((l + 1, 2 * ix + dx, 2 * iy + dy, 2 * iz + dz))
        leaves = _balance(leaves, base)
    return np.array(sorted(leaves), dtype=np.int32)


def orszag_tang(base=(8, 8, 2), nlevels=4, gamma=5.0 / 3.0, blocks=None, threshold=0.55, step=-0.1) -> Workload:
    """z-uniform Orszag-Tang vortex, periodic box (1, 1, base_z/base_x):
    rho = 25/(36 pi), p = 5/(12 pi), v = (-sin 2 pi y, sin 2 pi x, 0),
    B = (-sin 2 pi y, sin 4 pi x, 0)/sqrt(4 pi), psi = 0; HLL, CFL 0.4."""
    if blocks is None:
        blocks = orszag_tang_mesh(base, nlevels, threshold, step)
    s4 = 1.0 / np.sqrt(4.0 * np.pi)

    def prim(x, y, z, g, lev):
        one = np.ones(x.shape)
        return (25.0 / (36.0 * np.pi) * one, -np.sin(2 * np.pi * y), np.sin(2 * np.pi * x), 0.0 * one,
                5.0 / (12.0 * np.pi) * one, -s4 * np.sin(2 * np.pi * y), s4 * np.sin(4 * np.pi * x), 0.0 * one,
                0.0 * one)
    hi = (1.0, base[1] / base[0], base[2] / base[0])
    return _make(f"ot{16 * base[0]}_L{nlevels}", MHD, HLL, gamma, 0.4, blocks, (16, 16, 16), base, (0, 0, 0), hi,
                 nlevels, prim)


def dependent_levels_blocks() -> np.ndarray:
    """A 3-level 2:1 mesh over a 4^3 base in which one level-3 ghost slab is
    prolonged from a level-2 block whose own tangential ghosts are prolonged
    from level 1: level-1 blocks (1,1,1), (2,1,1), (2,0,1), (2,1,2) refined,
    then the level-2 block (4,2,3)."""
    b = uniform_blocks((4, 4, 4))
    rows = b.tolist()
    b = refine_blocks(b, [q for q, r in enumerate(rows) if tuple(r[1:]) in {(1, 1, 1), (2, 1, 1), (2, 0, 1), (2, 1, 2)}])
    rows = b.tolist()
    return refine_blocks(b, [q for q, r in enumerate(rows) if r[0] == 2 and tuple(r[1:]) == (4, 2, 3)])


# ---------------------------------------------------------------------------
# special relativistic hydrodynamics (SRHD, c = 1)

def srhd_advection(n=64, bn_long=16, bn_short=2, v=0.6, amp=0.3, p=1.0, gamma=5.0 / 3.0, axis=0,
                   riemann=LF) -> Workload:
    """A density wave rho = 1 + amp sin(2 pi x) carried at uniform speed v
    along `axis` at uniform pressure: a contact, so the exact solution is the
    advected profile.  Quasi-1-D periodic box of n cells along `axis`."""
    bn = [bn_short] * 3
    bn[axis] = bn_long
    base = [1, 1, 1]
    base[axis] = n // bn_long
    lo = (0.0, 0.0, 0.0)
    hi = [bn[d] * base[d] / n for d in range(3)]

    def prim(x, y, z, g, lev):
        c = (x, y, z)[axis]
        rho = 1.0 + amp * np.sin(2.0 * np.pi * c)
        vel = [np.zeros_like(rho)] * 3
        vel[axis] = np.full_like(rho, v)
        return (rho, *vel, np.full_like(rho, p))
    return _make(f"srhd_adv{n}", SRHD, riemann, gamma, 0.4, uniform_blocks(tuple(base)), tuple(bn), tuple(base),
                 lo, tuple(hi), 1, prim)


def srhd_smooth_random(blocks, base, max_level, seed=13, vmax=0.7, gamma=5.0 / 3.0, nmodes=3) -> Workload:
    """Smooth periodic SRHD state on any mesh: rho, p in [0.5, 2], |v| up to
    about vmax (Lorentz factors up to ~1.4)."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, 3, size=(5, nmodes, 3))
    ph = rng.random((5, nmodes)) * 2 * np.pi

    def field(x, y, z, f):
        out = np.zeros_like(x)
        for m in range(nmodes):
            out = out + np.sin(2 * np.pi * (k[f, m, 0] * x + k[f, m, 1] * y + k[f, m, 2] * z) + ph[f, m]) / nmodes
        return out

    def prim(x, y, z, g, lev):
        rho = 1.25 + 0.75 * field(x, y, z, 0)
        p = 1.25 + 0.75 * field(x, y, z, 4)
        v = [vmax / np.sqrt(3.0) * field(x, y, z, 1 + d) for d in range(3)]
        return (rho, *v, p)
    return _make("srhd_smooth", SRHD, LF, gamma, 0.4, blocks, (16, 16, 16), base, (0, 0, 0), (1, 1, 1), max_level,
                 prim)


def srhd_kelvin_helmholtz(n=256, seed=5, vshear=0.5, gamma=4.0 / 3.0) -> Workload:
    """Relativistic double shear layer: rho = 1, v_x = +-vshear (Lorentz
    factor 1.15 at 0.5), p = 1, v_y perturbation 0.01 sin(4 pi x) plus seeded
    noise 1e-3; periodic, n^3 cells in 16^3 blocks, LF."""
    def prim(x, y, z, g, lev):
        inside = np.abs(y - 0.5) < 0.25
        vx = np.where(inside, vshear, -vshear)
        vy = 0.01 * np.sin(4.0 * np.pi * x) + uniform(seed, g, 0, -1e-3, 1e-3)
        vz = uniform(seed, g, 1, -1e-3, 1e-3)
        return np.ones_like(x), vx, vy, vz, np.ones_like(x)
    base = (n // 16,) * 3
    return _make(f"srhd_kh{n}", SRHD, LF, gamma, 0.4, uniform_blocks(base), (16, 16, 16), base, (0, 0, 0),
                 (1, 1, 1), 1, prim)


def srhd_blast(blocks=None, base=(4, 4, 4), max_level=2, p_in=100.0, p_out=0.1, r0=0.15,
               gamma=4.0 / 3.0) -> Workload:
    """Relativistic spherical blast: rho = 1 at rest, p = p_in inside radius r0
    of the box centre, p_out outside; periodic unit box in 16^3 blocks, LF.
    The default mesh nests one finer level over the central half."""
    if blocks is None:
        blocks = nested_blocks(base, max_level)

    def prim(x, y, z, g, lev):
        r2 = ((x - 0.5) ** 2 + (y - 0.5) ** 2) + (z - 0.5) ** 2
        p = np.where(r2 < r0 * r0, p_in, p_out)
        return np.ones(x.shape), 0.0, 0.0, 0.0, p
    return _make("srhd_blast", SRHD, LF, gamma, 0.4, blocks, (16, 16, 16), tuple(base), (0, 0, 0), (1, 1, 1),
                 max_level, prim)


def srhd_fast_flow(blocks=None, base=(4, 4, 4), max_level=2, gamma=4.0 / 3.0) -> Workload:
    """A fast, relativistically cool flow like a jet's: v_x = 0.97 + 0.02
    sin 2pi(y + z), v_y = 0.05 sin 2pi z, v_z = 0.05 cos 2pi x (Lorentz factors
    3.2 to 8.2), rho = 1 + 0.5 sin 2pi x cos 2pi y, p = 0.1 + 0.05 sin 2pi(x - y);
    periodic unit box in 16^3 blocks, LF; by default one finer level over the
    central half."""
    if blocks is None:
        blocks = nested_blocks(base, max_level)

    def prim(x, y, z, g, lev):
        rho = 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
        vx = 0.97 + 0.02 * np.sin(2 * np.pi * (y + z))
        vy = 0.05 * np.sin(2 * np.pi * z)
        vz = 0.05 * np.cos(2 * np.pi * x)
        p = 0.1 + 0.05 * np.sin(2 * np.pi * (x - y))
        return rho, vx, vy, vz, p
    return _make("srhd_fast", SRHD, LF, gamma, 0.4, blocks, (16, 16, 16), tuple(base), (0, 0, 0), (1, 1, 1),
                 max_level, prim)


def srhd_double_tube(ncell=256, p_in=10.0, p_out=0.1, gamma=4.0 / 3.0, bn_long=16, bn_short=2) -> Workload:
    """Periodic relativistic double shock tube along x: rho = 1 at rest, p = p_in
    in [1/4, 3/4] and p_out outside; uniform across (one block of bn_short
    cells); LF."""
    base = (ncell // bn_long, 1, 1)

    def prim(x, y, z, g, lev):
        inside = (x > 0.25) & (x < 0.75)
        return np.ones(x.shape), 0.0, 0.0, 0.0, np.where(inside, p_in, p_out)
    return _make(f"srhd_dtube{ncell}", SRHD, LF, gamma, 0.4, uniform_blocks(base), (bn_long, bn_short, bn_short),
                 base, (0.0, 0.0, 0.0), (1.0, bn_short / ncell, bn_short / ncell), 1, prim)
