"""Parity metric between a HIP-path state and an oracle state (one step from
the same input): relative L-infinity per cell and variable.
  rho, e        : |dU| / |U_ref|
  momentum m_d  : |dm_d| / max(|m|, rho c_s)
so that near-zero momentum components are measured against the local flow
scale rather than against themselves."""
from __future__ import annotations

import numpy as np

TOL_FP64 = 1e-12


def parity_error(U, R, gamma):
    U = np.asarray(U, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    rho = R[:, 0]
    m = R[:, 1:4]
    e = R[:, 4]
    mm = np.sqrt((m * m).sum(axis=1))
    p = (gamma - 1.0) * (e - 0.5 * (m * m).sum(axis=1) / rho)
    cs = np.sqrt(gamma * np.abs(p) / rho)
    scale_m = np.maximum(mm, rho * cs)
    err = np.zeros(U.shape[1])
    err[0] = np.max(np.abs(U[:, 0] - rho) / np.abs(rho))
    for d in range(3):
        err[1 + d] = np.max(np.abs(U[:, 1 + d] - m[:, d]) / scale_m)
    err[4] = np.max(np.abs(U[:, 4] - e) / np.abs(e))
    return err


def parity_error_mhd(U, R, gamma):
    """MHD (nvar 9) analogue: rho, e pointwise relative; m against
    max(|m|, rho c_f); B against max(|B|, sqrt(rho) c_f); psi against
    max(|psi|, c_f |B|) with c_f = sqrt(a^2 + b^2) the largest fast speed."""
    U = np.asarray(U, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    rho = R[:, 0]
    m = R[:, 1:4]
    e = R[:, 4]
    B = R[:, 5:8]
    mm = np.sqrt((m * m).sum(axis=1))
    bb = (B * B).sum(axis=1)
    p = (gamma - 1.0) * (e - 0.5 * (m * m).sum(axis=1) / rho - 0.5 * bb)
    cf = np.sqrt((gamma * np.abs(p) + bb) / rho)
    err = np.zeros(9)
    err[0] = np.max(np.abs(U[:, 0] - rho) / np.abs(rho))
    sm = np.maximum(mm, rho * cf)
    sb = np.maximum(np.sqrt(bb), np.sqrt(rho) * cf)
    for d in range(3):
        err[1 + d] = np.max(np.abs(U[:, 1 + d] - m[:, d]) / sm)
        err[5 + d] = np.max(np.abs(U[:, 5 + d] - B[:, d]) / sb)
    err[4] = np.max(np.abs(U[:, 4] - e) / np.abs(e))
    err[8] = np.max(np.abs(U[:, 8] - R[:, 8]) / np.maximum(np.abs(R[:, 8]), cf * np.sqrt(bb)))
    return err


def parity_error_srhd(U, R):
    """SRHD (D, m, tau) analogue: D and tau pointwise relative; m_d against
    max(|m|, D + tau), the total energy density, which bounds |m| for every
    physical state."""
    U = np.asarray(U, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    D = R[:, 0]
    m = R[:, 1:4]
    tau = R[:, 4]
    scale_m = np.maximum(np.sqrt((m * m).sum(axis=1)), D + tau)
    err = np.zeros(U.shape[1])
    err[0] = np.max(np.abs(U[:, 0] - D) / np.abs(D))
    for d in range(3):
        err[1 + d] = np.max(np.abs(U[:, 1 + d] - m[:, d]) / scale_m)
    err[4] = np.max(np.abs(U[:, 4] - tau) / np.abs(tau))
    return err


def oracle_cfl_steps(w, steps):
    """The oracle's state and simulated time after `steps` CFL steps of
    workload w, each with the dt of its own state (as the device's CFL steps
    take theirs)."""
    from oracle.oracle import Oracle
    o = Oracle(w)
    t = 0.0
    for _ in range(steps):
        dt = o.dt()
        o.step(dt)
        t = t + dt
    return o.state(), t


def l1_rel(a, b):
    """sum |a - b| / sum |b| (the mixed-precision error measure)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).sum() / np.abs(b).sum())
