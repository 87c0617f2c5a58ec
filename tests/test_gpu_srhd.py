"""Special relativistic hydrodynamics (conserved D, m, tau; Lax-Friedrichs
flux) on an MI355X through the C-ABI, against the CPU oracle: the ghost fill
bitwise, the CFL dt to a few ulp, one step from the oracle's state to the
FP64 bar (with the paper's minmod / RK2 and van Leer / RK3 numerics), CFL
steps in a row, conservation, the FP32-flux variant, a full-size
shear-layer step, regrids, and batched requests equal to the same requests
alone."""
from __future__ import annotations

import dataclasses
import math
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2607_19277_amd import workloads as W
from parity import TOL_FP64, l1_rel, oracle_cfl_steps, parity_error_srhd

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
    "uniform": lambda: W.srhd_smooth_random(W.uniform_blocks((2, 2, 2)), (2, 2, 2), 1, seed=3),
    "nested2": lambda: W.srhd_smooth_random(W.nested_blocks((4, 4, 4), 2), (4, 4, 4), 2, seed=21),
    "dependent3": lambda: W.srhd_smooth_random(W.dependent_levels_blocks(), (4, 4, 4), 3, seed=17),
    "blast": lambda: W.srhd_blast(),
    "fast": lambda: W.srhd_fast_flow(),           # Lorentz factors 3.2 .. 8.2
    "tube": lambda: W.srhd_double_tube(256, bn_short=16),   # pressure ratio 100
}
SCHEMES = {
    "minmod_rk2": (W.MINMOD, 2),
    "vanleer_rk3": (W.VANLEER, 3),
}


@pytest.mark.parametrize("case", list(CASES))
def test_ghost_fill_matches_oracle_bitwise(agile, case):
    w = CASES[case]()
    _say(f"srhd ghosts {case} blocks={w.nblocks}")
    g = agile.Mesh.from_workload(w).read_ghosts()
    ref = Oracle(w).ghosts()
    assert g.shape == ref.shape
    bad = np.argwhere(g != ref)
    assert bad.size == 0, (bad[:5], g[tuple(bad[0])], ref[tuple(bad[0])])


# the device forms the SRHD signal with reciprocal-based arithmetic (the
# con2prim is an iteration either way): dt agrees with the oracle's to a few
# ulp, not bitwise
TOL_DT = 1e-13


@pytest.mark.parametrize("case", list(CASES))
def test_dt_matches_oracle(agile, case):
    w = CASES[case]()
    _say(f"srhd dt {case}")
    d_gpu = agile.Mesh.from_workload(w).dt()
    d_ref = Oracle(w).dt()
    assert abs(d_gpu - d_ref) <= TOL_DT * d_ref, (d_gpu, d_ref, (d_gpu - d_ref) / d_ref)


@pytest.mark.parametrize("case", ["nested2", "dependent3", "blast"])
def test_fused_signal_equals_dt_reduction_bitwise(agile, case):
    """The next step's dt from the signal maximum that the last RK stage and
    the flux correction form equals the dt reduction kernel's on the same
    state, bit for bit."""
    import torch
    w = CASES[case]()
    w.limiter, w.rk = W.VANLEER, 3
    m = agile.Mesh.from_workload(w)
    for _ in range(3):
        m.step_cfl(1)
        torch.cuda.synchronize()
        d = m.dt()
        m.step_cfl(1)
        assert m.last_dt() == d, (m.last_dt(), d)


@pytest.mark.parametrize("sch", list(SCHEMES))
@pytest.mark.parametrize("case", list(CASES))
def test_step_matches_oracle(agile, case, sch):
    w = CASES[case]()
    w.limiter, w.rk = SCHEMES[sch]
    _say(f"srhd step {case} {sch} blocks={w.nblocks}")
    o = Oracle(w)
    m = agile.Mesh.from_workload(w)
    for s in range(2):
        m.set_blocks(w.blocks, o.state())
        dt = o.dt()
        m.step(dt)
        o.step(dt)
        err = parity_error_srhd(m.readback(), o.state())
        _say(f"  step {s}: dt={dt:.6e} err={err.max():.3e}")
        assert err.max() <= TOL_FP64, (s, err)


@pytest.mark.parametrize("case", ["nested2", "blast", "fast", "tube"])
def test_consecutive_cfl_steps_match_oracle(agile, case):
    """Five CFL steps in a row on the GPU (dt from the device reduction,
    ghosts from the previous step's fill) against five oracle steps; the
    double shock tube runs 40 (its waves cross several cells)."""
    import torch
    w = CASES[case]()
    _say(f"srhd consecutive {case}")
    m = agile.Mesh.from_workload(w)
    o = Oracle(w)
    for k in range(40 if case == "tube" else 5):
        dt = o.dt()
        m.step_cfl(1)
        torch.cuda.synchronize()
        # the two states differ within the state bar after the first step
        assert abs(m.last_dt() - dt) <= 1e-12 * dt, (k, m.last_dt(), dt)
        dt = m.last_dt()
        o.step(dt)
        err = parity_error_srhd(m.readback(), o.state())
        _say(f"  step {k}: err={err.max():.3e}")
        assert err.max() <= TOL_FP64, (k, err)


def test_conservation_across_level_jumps(agile):
    w = CASES["blast"]()
    w.limiter, w.rk = W.VANLEER, 3
    m = agile.Mesh.from_workload(w)
    vol = np.array([w.dx(int(l)) ** 3 for l in w.blocks[:, 0]])

    def tot(U):
        return [(math.fsum((U[:, v] * vol[:, None, None, None]).ravel()),
                 math.fsum(np.abs(U[:, v] * vol[:, None, None, None]).ravel())) for v in range(5)]
    t0 = tot(w.U)
    m.step_cfl(4)
    t1 = tot(m.readback())
    for (a, na), (b, nb) in zip(t0, t1):
        assert abs(b - a) <= 1e-13 * max(na, nb), (a, b)


def test_fp32_flux_close_to_fp64(agile):
    w = W.srhd_kelvin_helmholtz(n=64)
    a = agile.Mesh.from_workload(w)
    b = agile.Mesh.from_workload(w, precision=agile.FP32_FLUX)
    dt = a.dt()
    for _ in range(5):
        a.step(dt)
        b.step(dt)
    Ua, Ub = a.readback(), b.readback()
    scale = np.abs(Ua).max(axis=(0, 2, 3, 4))
    scale[1:4] = np.sqrt((Ua[:, 1:4] ** 2).sum(axis=1)).max()
    err = np.abs(Ua - Ub).max(axis=(0, 2, 3, 4)) / scale
    _say(f"srhd fp32 vs fp64 after 5 steps: {err}")
    assert err.max() < 1e-5


def test_other_riemann_solvers_are_rejected(agile):
    w = CASES["uniform"]()
    for rs in (agile.HLL, agile.HLLC):
        w.riemann = rs
        with pytest.raises(agile.AgileError):
            agile.Mesh.from_workload(w)


def test_shear_layer_256_full_size(agile):
    """The 256^3 relativistic shear layer (4096 blocks of 16^3, LF, van Leer,
    RK3) in the benchmark's launch configuration: dt reduced on the device,
    one step against the oracle on the whole state."""
    w = W.srhd_kelvin_helmholtz(n=256)
    w.limiter, w.rk = W.VANLEER, 3
    _say(f"srhd kh256: {w.nblocks} blocks")
    o = Oracle(w)
    m = agile.Mesh.from_workload(w)
    dt = m.dt()
    assert abs(dt - o.dt()) <= TOL_DT * dt
    m.step_cfl(1)
    assert m.last_dt() == dt
    o.step(dt)
    err = parity_error_srhd(m.readback(), o.state())
    _say(f"  one step, dt={dt:.6e}: err per var {np.array2string(err, precision=2)}")
    assert err.max() <= TOL_FP64, err
    m.close()


REGRID = {
    # (workload, steps before the regrid, refine quantile)
    "smooth": (lambda: W.srhd_smooth_random(W.nested_blocks((4, 4, 4), 2), (4, 4, 4), 3, seed=21), 2, 0.8),
    "blast": (lambda: dataclasses.replace(W.srhd_blast(), max_level=3), 3, 0.85),
}


@pytest.mark.parametrize("case", list(REGRID))
def test_regrid_matches_oracle(agile, case):
    """Dynamic regrid on D after a few steps (the estimate bitwise, the
    decision and the transferred state equal to the oracle's), then a step on
    the new mesh.  The new fine cells of the blast sit across a relativistic
    shock, where only the prolongation of primitives keeps them physical."""
    from oracle import regrid as RG
    make, nsteps, qr = REGRID[case]
    w = make()
    m = agile.Mesh.from_workload(w)
    for _ in range(nsteps):
        m.step_cfl(1)
    U = m.readback()
    w1 = dataclasses.replace(w, U=U)
    err = m.error(0)
    assert np.array_equal(err, Oracle(w1).lohner(0, 0.01))
    refine, coarsen = float(np.quantile(err, qr)), float(np.quantile(err, 0.3))
    new_ref, R, P = RG.decide(w.blocks, err, w.base, w.max_level, refine, coarsen)
    _say(f"srhd regrid {case}: {w.nblocks} -> {len(new_ref)} blocks, refined {len(R)}, coarsened {len(P)}")
    assert R
    st = m.regrid(refine, coarsen, w.max_level, variable=0)
    assert st["new_blocks"] == len(new_ref)
    assert [tuple(r) for r in m.blocks().tolist()] == new_ref
    U_ref = Oracle(w1).remap(new_ref)
    assert np.array_equal(m.readback(), U_ref)
    w2 = dataclasses.replace(w, blocks=np.array(new_ref, dtype=np.int32), U=U_ref)
    o2 = Oracle(w2)
    dt = m.dt()
    m.step(dt)
    o2.step(dt)
    e = parity_error_srhd(m.readback(), o2.state())
    _say(f"  step after regrid: err={e.max():.3e}")
    assert e.max() <= TOL_FP64, e


@pytest.mark.parametrize("precision,graph", [(0, False), (0, True), (1, True)])
def test_batched_srhd_requests_equal_alone(agile, precision, graph):
    """SRHD requests served together (one launch per kernel class over all of
    them, graph replay and tuner on a stream): each result bitwise equal to
    the same request run alone, and within the FP64 bar of the oracle run for
    the same CFL steps (FP32 flux: 1e-5 in relative L1 of D and tau)."""
    import torch
    ws = {k: CASES[k]() for k in ("uniform", "nested2", "blast", "tube")}
    steps = {"uniform": 3, "nested2": 5, "blast": 2, "tube": 4}
    s = torch.cuda.Stream() if graph else None
    b = agile.Batch(physics=W.SRHD, riemann=W.LF, precision=precision, budget_bytes=1 << 30, use_graph=graph,
                    autotune=graph, stream=s)
    for tag, (name, w) in enumerate(ws.items()):
        b.submit(w, steps[name], tag)
    done = {}
    for _ in range(20):
        info = b.tick()
        for tag in range(len(ws)):
            if tag not in done and b.status(tag)[0] == agile.REQ_FINISHED:
                done[tag] = b.result(tag)
        if len(done) == len(ws):
            break
    assert len(done) == len(ws), info
    for tag, (name, w) in enumerate(ws.items()):
        U, n, t = done[tag]
        m = agile.Mesh.from_workload(w, precision=precision)
        m.step_cfl(steps[name])
        assert n == steps[name]
        assert np.array_equal(U, m.readback()), name
        assert t == m.time(), (name, t, m.time())
        m.close()
        R, t_ref = oracle_cfl_steps(w, steps[name])
        assert abs(t - t_ref) <= (1e-12 if precision == 0 else 1e-6) * t_ref, (name, t, t_ref)
        if precision == 0:
            err = parity_error_srhd(U, R).max()
            assert err <= TOL_FP64, (name, err)
        else:
            err = max(l1_rel(U[:, 0], R[:, 0]), l1_rel(U[:, 4], R[:, 4]))
            assert err <= 1e-5, (name, err)
        _say(f"srhd batch {name}: {n} steps bitwise equal alone, oracle err {err:.2e}")


def test_nonphysical_state_is_reported(agile):
    """A cell with |m| > tau + D (superluminal, no primitives) is reported by
    the dt reduction, and a step on it leaves the mesh in the error state."""
    w = CASES["uniform"]()
    U = w.U.copy()
    U[3, 1, 5, 6, 7] = 2.0 * (U[3, 0, 5, 6, 7] + U[3, 4, 5, 6, 7])
    m = agile.Mesh.from_workload(w, U=U)
    with pytest.raises(agile.AgileError) as e:
        m.dt()
    assert e.value.code == agile.ENONPHYSICAL
    with pytest.raises(agile.AgileError) as e:
        m.step(1e-4)
    assert e.value.code == agile.ESTATE
