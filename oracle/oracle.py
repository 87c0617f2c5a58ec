"""ctypes wrapper around the plain FP64 CPU oracle (agile_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "agile_oracle.c")
LIB = os.environ.get("AGILE_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC", "-Wall"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (strict IEEE, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, ip, ip, dp, dp,
                                 C.c_int, C.c_int, ip, C.c_char_p, C.c_int]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_scheme.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc_nvar.argtypes = [C.c_void_p]
        L.orc_set_state.argtypes = [C.c_void_p, dp]
        L.orc_get_state.argtypes = [C.c_void_p, dp]
        L.orc_fill_ghosts.argtypes = [C.c_void_p]
        L.orc_get_ghosts.argtypes = [C.c_void_p, dp]
        L.orc_max_speed.argtypes = [C.c_void_p, dp, dp]
        L.orc_dt.argtypes = [C.c_void_p]
        L.orc_dt.restype = C.c_double
        L.orc_rhs.argtypes = [C.c_void_p, dp]
        L.orc_step.argtypes = [C.c_void_p, C.c_double]
        L.orc_face_flux.argtypes = [C.c_void_p, dp, dp, C.c_int, C.c_double, dp]
        L.orc_get_ch.argtypes = [C.c_void_p]
        L.orc_get_ch.restype = C.c_double
        L.orc_lohner.argtypes = [C.c_void_p, C.c_int, C.c_double, dp]
        L.orc_cons_to_prim.argtypes = [C.c_void_p, C.c_long, dp, dp]
        L.orc_srhd_newton_steps.argtypes = [C.c_void_p, C.c_long, dp, C.POINTER(C.c_int)]
        L.orc_remap.argtypes = [C.c_void_p, C.c_long, ip, dp]
        L.orc_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleError(RuntimeError):
    pass


class Oracle:
    """One mesh held by the oracle, built from a workloads.Workload."""

    def __init__(self, w, U=None):
        L = lib()
        self.w = w
        blocks = np.ascontiguousarray(w.blocks, dtype=np.int32)
        bn = (C.c_int * 3)(*w.bn)
        base = (C.c_int * 3)(*w.base)
        lo = (C.c_double * 3)(*w.lo)
        hi = (C.c_double * 3)(*w.hi)
        err = C.create_string_buffer(256)
        h = L.orc_create(w.physics, w.riemann, w.gamma, w.cfl, w.glm_alpha, bn, base, lo, hi, w.max_level,
                         blocks.shape[0], blocks.ctypes.data_as(C.POINTER(C.c_int)), err, 256)
        if not h:
            raise OracleError(err.value.decode())
        if L.orc_set_scheme(h, int(getattr(w, "limiter", 0)), int(getattr(w, "rk", 2))) != 0:
            L.orc_destroy(h)
            raise OracleError("bad limiter / Runge-Kutta stages")
        self.h = C.c_void_p(h)
        self.nvar = L.orc_nvar(self.h)
        self.n = blocks.shape[0]
        self.shape = (self.n, self.nvar, w.bn[2], w.bn[1], w.bn[0])
        self.set_state(w.U if U is None else U)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def set_state(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == self.shape, (U.shape, self.shape)
        lib().orc_set_state(self.h, _dp(U))

    def state(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float64)
        lib().orc_get_state(self.h, _dp(out))
        return out

    def fill_ghosts(self):
        lib().orc_fill_ghosts(self.h)

    def ghosts(self) -> np.ndarray:
        """[n, 6 faces, nvar, 2*bn*bn] face ghosts (fills first). Cubic blocks only."""
        bn = self.w.bn
        assert bn[0] == bn[1] == bn[2]
        self.fill_ghosts()
        out = np.empty((self.n, 6, self.nvar, 2 * bn[0] * bn[0]), dtype=np.float64)
        lib().orc_get_ghosts(self.h, _dp(out))
        return out

    def max_speed(self):
        s = np.zeros(1)
        c = np.zeros(1)
        e = lib().orc_max_speed(self.h, _dp(s), _dp(c))
        if e:
            raise OracleError(f"non-physical state ({e})")
        return float(s[0]), float(c[0])

    def dt(self) -> float:
        d = lib().orc_dt(self.h)
        if d < 0:
            raise OracleError(f"non-physical state ({d})")
        return d

    def rhs(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float64)
        e = lib().orc_rhs(self.h, _dp(out))
        if e:
            raise OracleError(f"rhs failed ({e})")
        return out

    def step(self, dt: float):
        e = lib().orc_step(self.h, float(dt))
        if e:
            raise OracleError(f"step failed ({e})")

    def ch(self) -> float:
        return lib().orc_get_ch(self.h)

    def lohner(self, v: int = 0, eps: float = 0.01) -> np.ndarray:
        """Loehner error indicator of variable v: per block the maximum over
        its cells (fills the ghosts first)."""
        out = np.zeros(self.n)
        if lib().orc_lohner(self.h, int(v), float(eps), _dp(out)) != 0:
            raise OracleError("bad estimator arguments")
        return out

    def remap(self, blocks) -> np.ndarray:
        """State of a new block list [(level, bx, by, bz)] sampled from this
        mesh (copy, prolongation or restriction by point location)."""
        b = np.ascontiguousarray(blocks, dtype=np.int32).reshape(-1, 4)
        out = np.zeros((b.shape[0], self.nvar, self.w.bn[2], self.w.bn[1], self.w.bn[0]))
        if lib().orc_remap(self.h, b.shape[0], b.ctypes.data_as(C.POINTER(C.c_int)), _dp(out)) != 0:
            raise OracleError("block outside the domain or level range")
        return out

    def cons_to_prim(self, U) -> np.ndarray:
        """Primitives of conserved states [n, nvar] (SRHD: rho, Gamma v, p)."""
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(-1, self.nvar)
        w = np.zeros_like(U)
        if lib().orc_cons_to_prim(self.h, U.shape[0], _dp(U), _dp(w)) != 0:
            raise OracleError("non-physical state")
        return w

    def srhd_newton_steps(self, U) -> np.ndarray:
        """Newton steps of the SRHD con2prim for conserved states [n, 5]."""
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(-1, 5)
        out = np.zeros(U.shape[0], dtype=np.int32)
        if lib().orc_srhd_newton_steps(self.h, U.shape[0], _dp(U), out.ctypes.data_as(C.POINTER(C.c_int))) != 0:
            raise OracleError("not an SRHD mesh")
        return out

    def face_flux(self, wL, wR, d, ch=1.0):
        wL = np.ascontiguousarray(wL, dtype=np.float64)
        wR = np.ascontiguousarray(wR, dtype=np.float64)
        F = np.zeros(self.nvar)
        lib().orc_face_flux(self.h, _dp(wL), _dp(wR), int(d), float(ch), _dp(F))
        return F


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int):
    lib().orc_set_threads(int(n))
