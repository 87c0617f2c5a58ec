"""Python binding of the MI355X block-AMR library (include/agile.h).

Argument marshalling only: every step of the update runs in the HIP kernels
of libagile.so.  Device arrays are torch CUDA (ROCm) tensors; streams are torch
streams (or raw hipStream_t handles).  The library must have been built
in-tree (``python -m paper_2607_19277_amd.build`` or ``__graft_entry__.build()``);
there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("AGILE_LIB") or os.path.join(HERE, "libagile.so")   # AGILE_LIB: another build

EULER, MHD_GLM, SRHD = 0, 1, 2
HLL, HLLC, LF = 0, 1, 2
MINMOD, VANLEER = 0, 1
FP64, FP32_FLUX = 0, 1

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENONPHYSICAL = 0, -1, -2, -3, -4, -5

EXPORTS = ["agile_mesh_create", "agile_set_blocks", "agile_fill_ghosts", "agile_dt", "agile_step",
           "agile_step_cfl", "agile_last_dt", "agile_readback", "agile_read_ghosts", "agile_plan",
           "agile_mesh_info", "agile_mesh_destroy", "agile_strerror", "agile_last_error", "agile_profile",
           "agile_profile_read", "agile_mesh_set_option", "agile_mesh_get_option", "agile_mesh_tune",
           "agile_mesh_time", "agile_batch_create", "agile_batch_capacity", "agile_batch_submit",
           "agile_batch_tick", "agile_batch_status", "agile_batch_result", "agile_batch_cancel",
           "agile_batch_destroy", "agile_batch_last_error", "agile_mesh_error", "agile_regrid_decide",
           "agile_mesh_regrid", "agile_mesh_blocks", "agile_mesh_regrid_noalloc", "agile_copy_probe",
           "agile_batch_regrid", "agile_batch_blocks"]

K_STAGE, K_FILL, K_REFLUX, K_DT = 0, 1, 2, 3
PROFILE_ALL, PROFILE_KEEP = 15, 16
OPT_GRAPH, OPT_KSLAB, OPT_XCD, OPT_KSLAB_LAST, OPT_XCD_LAST = 0, 1, 2, 3, 4
REQ_UNKNOWN, REQ_QUEUED, REQ_RUNNING, REQ_FINISHED = 0, 1, 2, 3


class AgileConfig(C.Structure):
    _fields_ = [("physics", C.c_int), ("riemann", C.c_int), ("precision", C.c_int),
                ("gamma", C.c_double), ("cfl", C.c_double), ("glm_alpha", C.c_double),
                ("block_n", C.c_int), ("nghost", C.c_int), ("base_blocks", C.c_int * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("max_level", C.c_int),
                ("stream", C.c_void_p), ("limiter", C.c_int), ("rk_stages", C.c_int),
                ("dev_pool", C.c_void_p), ("dev_pool_bytes", C.c_size_t)]


class AgilePlanStats(C.Structure):
    _fields_ = [("nblocks", C.c_int64), ("same_level_faces", C.c_int64), ("restrict_tasks", C.c_int64),
                ("prolong_tasks", C.c_int64), ("reflux_blocks", C.c_int64), ("flux_registers", C.c_int64),
                ("levels", C.c_int), ("nvar", C.c_int), ("device_bytes", C.c_int64),
                ("prolong_launches", C.c_int), ("fused_correction", C.c_int)]


class AgileRegridParams(C.Structure):
    _fields_ = [("variable", C.c_int), ("max_level", C.c_int), ("refine", C.c_double), ("coarsen", C.c_double),
                ("eps", C.c_double)]


class AgileRegridStats(C.Structure):
    _fields_ = [("old_blocks", C.c_int64), ("new_blocks", C.c_int64), ("refined", C.c_int64),
                ("coarsened", C.c_int64)]


class AgileBatchConfig(C.Structure):
    _fields_ = [("physics", C.c_int), ("riemann", C.c_int), ("precision", C.c_int),
                ("budget_bytes", C.c_int64), ("max_meshes", C.c_int), ("use_graph", C.c_int),
                ("autotune", C.c_int), ("stream", C.c_void_p), ("dev_pool", C.c_void_p),
                ("dev_pool_bytes", C.c_size_t), ("max_active_blocks", C.c_int64)]


class AgileTickInfo(C.Structure):
    _fields_ = [("queued", C.c_int64), ("resident", C.c_int64), ("active", C.c_int64), ("admitted", C.c_int64),
                ("finished", C.c_int64), ("active_blocks", C.c_int64), ("free_blocks", C.c_int64),
                ("admit_ms", C.c_double), ("build_ms", C.c_double), ("graph_builds", C.c_int64)]


class AgileError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"agile error {code} ({msg})")
        self.code = code


_lib = None


def lib() -> C.CDLL:
    """Load libagile.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -m paper_2607_19277_amd.build)")
        L = C.CDLL(LIB_PATH)
        vp, i64, dp = C.c_void_p, C.c_int64, C.POINTER(C.c_double)
        L.agile_mesh_create.argtypes = [C.POINTER(AgileConfig), C.POINTER(vp)]
        L.agile_set_blocks.argtypes = [vp, i64, vp, vp, C.c_int]
        L.agile_fill_ghosts.argtypes = [vp]
        L.agile_dt.argtypes = [vp, dp]
        L.agile_step.argtypes = [vp, C.c_double]
        L.agile_step_cfl.argtypes = [vp, C.c_int]
        L.agile_last_dt.argtypes = [vp, dp]
        L.agile_readback.argtypes = [vp, vp, i64, C.c_int]
        L.agile_read_ghosts.argtypes = [vp, vp, i64, C.c_int]
        L.agile_plan.argtypes = [C.POINTER(AgileConfig), i64, vp, C.POINTER(AgilePlanStats), C.c_char_p, C.c_int]
        L.agile_mesh_error.argtypes = [vp, C.c_int, C.c_double, vp]
        L.agile_regrid_decide.argtypes = [C.POINTER(AgileConfig), i64, vp, vp, C.POINTER(AgileRegridParams), i64, vp,
                                          C.POINTER(i64), C.POINTER(AgileRegridStats)]
        L.agile_mesh_regrid.argtypes = [vp, C.POINTER(AgileRegridParams), C.POINTER(AgileRegridStats)]
        L.agile_mesh_regrid_noalloc.argtypes = [vp, C.POINTER(AgileRegridParams), C.POINTER(AgileRegridStats)]
        L.agile_mesh_blocks.argtypes = [vp, i64, vp, C.POINTER(i64)]
        L.agile_mesh_info.argtypes = [vp, C.POINTER(i64), C.POINTER(C.c_int)]
        L.agile_copy_probe.argtypes = [vp, vp, C.c_size_t, vp]
        L.agile_profile.argtypes = [vp, C.c_int]
        L.agile_profile_read.argtypes = [vp, C.c_int, dp, C.POINTER(i64)]
        L.agile_mesh_set_option.argtypes = [vp, C.c_int, C.c_int]
        L.agile_mesh_get_option.argtypes = [vp, C.c_int, C.POINTER(C.c_int)]
        L.agile_mesh_tune.argtypes = [vp]
        L.agile_mesh_time.argtypes = [vp, dp]
        L.agile_batch_create.argtypes = [C.POINTER(AgileBatchConfig), C.POINTER(vp)]
        L.agile_batch_capacity.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
        L.agile_batch_submit.argtypes = [vp, C.POINTER(AgileConfig), i64, vp, vp, C.c_int, i64, C.c_uint64]
        L.agile_batch_tick.argtypes = [vp, C.POINTER(AgileTickInfo)]
        L.agile_batch_status.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int), C.POINTER(i64)]
        L.agile_batch_result.argtypes = [vp, C.c_uint64, vp, i64, C.c_int, C.POINTER(i64), dp]
        L.agile_batch_cancel.argtypes = [vp, C.c_uint64]
        L.agile_batch_regrid.argtypes = [vp, C.c_uint64, C.POINTER(AgileRegridParams), C.POINTER(AgileRegridStats)]
        L.agile_batch_blocks.argtypes = [vp, C.c_uint64, i64, vp, C.POINTER(i64)]
        L.agile_batch_destroy.argtypes = [vp]
        L.agile_batch_destroy.restype = None
        L.agile_batch_last_error.argtypes = [vp]
        L.agile_batch_last_error.restype = C.c_char_p
        L.agile_mesh_destroy.argtypes = [vp]
        L.agile_mesh_destroy.restype = None
        L.agile_strerror.argtypes = [C.c_int]
        L.agile_strerror.restype = C.c_char_p
        L.agile_last_error.argtypes = [vp]
        L.agile_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                return torch.cuda.current_stream().cuda_stream
        except ImportError:
            pass
        return 0
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


def _pool_args(pool):
    """(pointer, bytes) of a caller-owned device pool: a contiguous CUDA
    (ROCm) tensor of any dtype, 256-byte aligned; None: no pool."""
    if pool is None:
        return None, 0
    if not _is_device(pool) or not pool.is_contiguous():
        raise ValueError("dev_pool must be a contiguous device tensor")
    if pool.data_ptr() % 256:
        raise ValueError("dev_pool must be 256-byte aligned")
    return pool.data_ptr(), pool.numel() * pool.element_size()


def make_config(physics=EULER, riemann=HLLC, precision=FP64, gamma=5.0 / 3.0, cfl=0.4, glm_alpha=0.5,
                base_blocks=(1, 1, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), max_level=1, stream=None,
                limiter=MINMOD, rk_stages=2, pool=None, block_n=16):
    cfg = AgileConfig()
    cfg.physics, cfg.riemann, cfg.precision = int(physics), int(riemann), int(precision)
    cfg.gamma, cfg.cfl, cfg.glm_alpha = float(gamma), float(cfl), float(glm_alpha)
    cfg.block_n, cfg.nghost = int(block_n), 2
    cfg.base_blocks = (C.c_int * 3)(*[int(b) for b in base_blocks])
    cfg.lo = (C.c_double * 3)(*[float(x) for x in lo])
    cfg.hi = (C.c_double * 3)(*[float(x) for x in hi])
    cfg.max_level = int(max_level)
    cfg.stream = C.c_void_p(_stream_handle(stream) or None)
    cfg.limiter, cfg.rk_stages = int(limiter), int(rk_stages)
    ptr, nbytes = _pool_args(pool)
    cfg.dev_pool, cfg.dev_pool_bytes = C.c_void_p(ptr), int(nbytes)
    return cfg


def _blocks_array(blocks) -> np.ndarray:
    b = np.ascontiguousarray(np.asarray(blocks, dtype=np.int32))
    if b.ndim != 2 or b.shape[1] != 4:
        raise ValueError("blocks must be an int array [n, 4] of (level, ix, iy, iz)")
    return b


def regrid_params(refine, coarsen, max_level, variable=0, eps=0.01) -> AgileRegridParams:
    return AgileRegridParams(int(variable), int(max_level), float(refine), float(coarsen), float(eps))


def regrid_decide(blocks, err, refine, coarsen, finest, variable=0, eps=0.01, **cfg_kw):
    """Host-only refine / coarsen decision, refining up to level `finest`
    (cfg_kw: the mesh config, e.g. base_blocks, max_level): (new sorted
    blocks [m, 4], stats)."""
    b = _blocks_array(blocks)
    e = np.ascontiguousarray(err, dtype=np.float64)
    if e.shape != (b.shape[0],):
        raise ValueError("one estimate per block")
    cfg = make_config(**cfg_kw)
    p = regrid_params(refine, coarsen, finest, variable, eps)
    cap = 8 * b.shape[0] + 8
    out = np.zeros((cap, 4), dtype=np.int32)
    n = C.c_int64()
    st = AgileRegridStats()
    rc = lib().agile_regrid_decide(C.byref(cfg), b.shape[0], b.ctypes.data, e.ctypes.data, C.byref(p), cap,
                                   out.ctypes.data, C.byref(n), C.byref(st))
    if rc != OK:
        raise AgileError(rc, "regrid decision rejected its input")
    return out[:n.value].copy(), {f: getattr(st, f) for f, _ in AgileRegridStats._fields_}


def copy_probe(dst, src, stream=None):
    """Streaming copy of device tensor src into dst (same byte size, a
    multiple of 16): the library's bandwidth probe, asynchronous on `stream`."""
    nbytes = src.numel() * src.element_size()
    if (not _is_device(dst) or not _is_device(src) or not dst.is_contiguous() or not src.is_contiguous()
            or dst.numel() * dst.element_size() != nbytes):
        raise ValueError("copy_probe: contiguous device tensors of the same byte size")
    rc = lib().agile_copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, C.c_void_p(_stream_handle(stream) or None))
    if rc != OK:
        raise AgileError(rc, lib().agile_strerror(rc).decode())


def plan(blocks, **cfg_kw) -> dict:
    """Validate a block list on the host (no GPU) and return the table sizes."""
    b = _blocks_array(blocks)
    cfg = make_config(**cfg_kw)
    st = AgilePlanStats()
    msg = C.create_string_buffer(512)
    rc = lib().agile_plan(C.byref(cfg), b.shape[0], b.ctypes.data, C.byref(st), msg, 512)
    if rc != OK:
        raise AgileError(rc, msg.value.decode())
    return {f: getattr(st, f) for f, _ in AgilePlanStats._fields_}


def _is_device(a) -> bool:
    return hasattr(a, "data_ptr") and getattr(a, "is_cuda", False)


def _device_out(out, shape, what):
    """A device output must be a contiguous float64 tensor of exactly `shape`."""
    import torch
    if tuple(out.shape) != tuple(shape) or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError(f"{what}: device output must be a contiguous float64 tensor {list(shape)}")
    return out


def _host_out(out, shape, what):
    """A host output (None: a new array) must be a C-contiguous, writable
    float64 ndarray of exactly `shape`."""
    if out is None:
        return np.empty(shape, dtype=np.float64)
    if (not isinstance(out, np.ndarray) or out.dtype != np.float64 or out.shape != tuple(shape)
            or not out.flags.c_contiguous or not out.flags.writeable):
        raise ValueError(f"{what}: host output must be a C-contiguous writable float64 array {list(shape)}")
    return out


class Mesh:
    """One mesh on the GPU.  See include/agile.h for the semantics of each call."""

    def __init__(self, physics=EULER, riemann=HLLC, precision=FP64, gamma=5.0 / 3.0, cfl=0.4, glm_alpha=0.5,
                 base_blocks=(1, 1, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), max_level=1, stream=None,
                 limiter=MINMOD, rk_stages=2, pool=None, block_n=16):
        """pool: optional device tensor whose memory holds every device array
        of the mesh (at least plan(...)["device_bytes"] bytes); it is kept
        referenced until close().  block_n: cells per block edge, 16, 32 or 64."""
        self._lib = lib()
        self.cfg = make_config(physics, riemann, precision, gamma, cfl, glm_alpha, base_blocks, lo, hi, max_level,
                               stream, limiter, rk_stages, pool, block_n)
        self._pool = pool
        self.bn = int(block_n)
        self.nvar = 9 if physics == MHD_GLM else 5
        h = C.c_void_p()
        rc = self._lib.agile_mesh_create(C.byref(self.cfg), C.byref(h))
        if rc != OK:
            raise AgileError(rc, self._lib.agile_strerror(rc).decode())
        self.h = h
        self.n = 0

    @classmethod
    def from_workload(cls, w, precision=FP64, stream=None, U=None, pool=None):
        m = cls(w.physics, w.riemann, precision, w.gamma, w.cfl, w.glm_alpha, w.base, w.lo, w.hi, w.max_level,
                stream, getattr(w, "limiter", MINMOD), getattr(w, "rk", 2), pool, w.bn[0])
        m.set_blocks(w.blocks, w.U if U is None else U)
        return m

    def _check(self, rc):
        if rc != OK:
            msg = self._lib.agile_last_error(self.h).decode() if self.h else ""
            raise AgileError(rc, msg or self._lib.agile_strerror(rc).decode())

    def set_blocks(self, blocks, U):
        b = _blocks_array(blocks)
        n = b.shape[0]
        B = self.bn
        if _is_device(U):
            if tuple(U.shape) != (n, self.nvar, B, B, B) or not U.is_contiguous() or str(U.dtype) != "torch.float64":
                raise ValueError(f"device state must be a contiguous float64 tensor [n, nvar, {B}, {B}, {B}]")
            self._check(self._lib.agile_set_blocks(self.h, n, b.ctypes.data, U.data_ptr(), 1))
        else:
            A = np.ascontiguousarray(U, dtype=np.float64)
            if A.shape != (n, self.nvar, B, B, B):
                raise ValueError(f"state must be [n, nvar, {B}, {B}, {B}]")
            self._check(self._lib.agile_set_blocks(self.h, n, b.ctypes.data, A.ctypes.data, 0))
        self.n = n

    def fill_ghosts(self):
        self._check(self._lib.agile_fill_ghosts(self.h))

    def dt(self) -> float:
        d = C.c_double()
        self._check(self._lib.agile_dt(self.h, C.byref(d)))
        return d.value

    def last_dt(self) -> float:
        d = C.c_double()
        self._check(self._lib.agile_last_dt(self.h, C.byref(d)))
        return d.value

    def step(self, dt: float):
        self._check(self._lib.agile_step(self.h, float(dt)))

    def step_cfl(self, nsteps: int = 1):
        self._check(self._lib.agile_step_cfl(self.h, int(nsteps)))

    def readback(self, out=None):
        shape = (self.n, self.nvar, self.bn, self.bn, self.bn)
        if out is not None and _is_device(out):
            _device_out(out, shape, "readback")
            self._check(self._lib.agile_readback(self.h, out.data_ptr(), out.numel(), 1))
            return out
        A = _host_out(out, shape, "readback")
        self._check(self._lib.agile_readback(self.h, A.ctypes.data, A.size, 0))
        return A

    def read_ghosts(self, out=None):
        shape = (self.n, 6, self.nvar, 512)
        if out is not None and _is_device(out):
            _device_out(out, shape, "read_ghosts")
            self._check(self._lib.agile_read_ghosts(self.h, out.data_ptr(), out.numel(), 1))
            return out
        A = _host_out(out, shape, "read_ghosts")
        self._check(self._lib.agile_read_ghosts(self.h, A.ctypes.data, A.size, 0))
        return A

    def error(self, variable: int = 0, eps: float = 0.01) -> np.ndarray:
        """Per-block Loehner estimate of the current state (caller's order)."""
        out = np.empty(self.n, dtype=np.float64)
        self._check(self._lib.agile_mesh_error(self.h, int(variable), float(eps), out.ctypes.data))
        return out

    def regrid(self, refine, coarsen, max_level, variable: int = 0, eps: float = 0.01) -> dict:
        """Estimate, decide and transfer the state to the new leaves on the
        device; the mesh then holds the new sorted block list."""
        p = regrid_params(refine, coarsen, max_level, variable, eps)
        st = AgileRegridStats()
        self._check(self._lib.agile_mesh_regrid(self.h, C.byref(p), C.byref(st)))
        self.n = int(st.new_blocks)
        return {f: getattr(st, f) for f, _ in AgileRegridStats._fields_}

    def regrid_noalloc(self, refine, coarsen, max_level, variable: int = 0, eps: float = 0.01) -> dict:
        """regrid() without any device allocation: the new mesh must fit in
        the mesh's device memory (AGILE_ENOMEM otherwise, mesh unchanged)."""
        p = regrid_params(refine, coarsen, max_level, variable, eps)
        st = AgileRegridStats()
        rc = self._lib.agile_mesh_regrid_noalloc(self.h, C.byref(p), C.byref(st))
        if rc != OK:
            raise AgileError(rc, self._lib.agile_last_error(self.h).decode() or self._lib.agile_strerror(rc).decode())
        self.n = int(st.new_blocks)
        return {f: getattr(st, f) for f, _ in AgileRegridStats._fields_}

    def blocks(self) -> np.ndarray:
        out = np.zeros((self.n, 4), dtype=np.int32)
        n = C.c_int64()
        self._check(self._lib.agile_mesh_blocks(self.h, self.n, out.ctypes.data, C.byref(n)))
        return out[:n.value]

    def set_option(self, option: int, value: int):
        self._check(self._lib.agile_mesh_set_option(self.h, int(option), int(value)))

    def get_option(self, option: int) -> int:
        v = C.c_int()
        self._check(self._lib.agile_mesh_get_option(self.h, int(option), C.byref(v)))
        return v.value

    def tune(self):
        """Pick the fastest stage-kernel shapes (bitwise-identical results):
        returns (kslab, xcd) of the first and middle stages and (kslab, xcd)
        of the last stage of a step."""
        self._check(self._lib.agile_mesh_tune(self.h))
        return (self.get_option(OPT_KSLAB), self.get_option(OPT_XCD),
                self.get_option(OPT_KSLAB_LAST), self.get_option(OPT_XCD_LAST))

    def time(self) -> float:
        t = C.c_double()
        self._check(self._lib.agile_mesh_time(self.h, C.byref(t)))
        return t.value

    def profile(self, enable=True, kinds=None, keep=False):
        """Start (and clear) or stop per-kernel event timing on the mesh's stream:
        every kernel class, or those listed in `kinds` (K_STAGE, K_FILL, ...).
        keep: only switch the timed classes (no wait, totals kept), to time
        some steps of a loop."""
        mask = 0
        if enable:
            mask = PROFILE_ALL if kinds is None else sum(1 << int(k) for k in set(kinds))
        self._check(self._lib.agile_profile(self.h, mask | (PROFILE_KEEP if keep else 0)))

    def profile_read(self, kind: int = K_STAGE):
        """(total kernel ms, launches) of one kernel class since the last clear."""
        ms = C.c_double()
        n = C.c_int64()
        self._check(self._lib.agile_profile_read(self.h, int(kind), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "h", None):
            self._lib.agile_mesh_destroy(self.h)
            self.h = None
        self._pool = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched serving of independent meshes on one GPU (see include/agile.h)."""

    def __init__(self, physics=EULER, riemann=HLLC, precision=FP64, budget_bytes=0, max_meshes=1024,
                 use_graph=False, autotune=False, stream=None, pool=None, max_active_blocks=0):
        """pool: optional device tensor that holds the whole block pool (then
        budget_bytes is ignored); kept referenced until close().
        max_active_blocks: step-latency budget of admission (0: none)."""
        self._lib = lib()
        cfg = AgileBatchConfig()
        cfg.physics, cfg.riemann, cfg.precision = int(physics), int(riemann), int(precision)
        cfg.budget_bytes, cfg.max_meshes = int(budget_bytes), int(max_meshes)
        cfg.use_graph, cfg.autotune = int(bool(use_graph)), int(bool(autotune))
        cfg.stream = C.c_void_p(_stream_handle(stream) or None)
        ptr, nbytes = _pool_args(pool)
        cfg.dev_pool, cfg.dev_pool_bytes = C.c_void_p(ptr), int(nbytes)
        cfg.max_active_blocks = int(max_active_blocks)
        self._pool = pool
        self.physics, self.riemann, self.precision = physics, riemann, precision
        h = C.c_void_p()
        rc = self._lib.agile_batch_create(C.byref(cfg), C.byref(h))
        if rc != OK:
            raise AgileError(rc, self._lib.agile_strerror(rc).decode())
        self.h = h
        self.sizes = {}
        self._pending = {}   # tag -> device initial state, kept alive until admission

    def _check(self, rc):
        if rc != OK:
            msg = self._lib.agile_batch_last_error(self.h).decode() if self.h else ""
            raise AgileError(rc, msg or self._lib.agile_strerror(rc).decode())

    def capacity(self):
        cap, free = C.c_int64(), C.c_int64()
        self._check(self._lib.agile_batch_capacity(self.h, C.byref(cap), C.byref(free)))
        return cap.value, free.value

    def submit(self, w, nsteps: int, tag: int, U=None):
        """Queue workload `w` (workloads.Workload) for nsteps CFL steps.  U (default
        w.U) is a host array or a device tensor; a device tensor is referenced
        until the request is admitted."""
        cfg = make_config(self.physics, self.riemann, self.precision, w.gamma, w.cfl, w.glm_alpha, w.base, w.lo,
                          w.hi, w.max_level, None, getattr(w, "limiter", MINMOD), getattr(w, "rk", 2))
        b = _blocks_array(w.blocks)
        src = w.U if U is None else U
        shape = (b.shape[0], 5, 16, 16, 16)
        if _is_device(src):
            import torch
            if tuple(src.shape) != shape or src.dtype != torch.float64 or not src.is_contiguous():
                raise ValueError("device state must be a contiguous float64 [n, 5, 16, 16, 16] tensor")
            ptr, on_dev, A = src.data_ptr(), 1, src
        else:
            A = np.ascontiguousarray(src, dtype=np.float64)
            if A.shape != shape:
                raise ValueError("state must be [n, 5, 16, 16, 16]")
            ptr, on_dev = A.ctypes.data, 0
        self._check(self._lib.agile_batch_submit(self.h, C.byref(cfg), b.shape[0], b.ctypes.data, C.c_void_p(ptr),
                                                 on_dev, int(nsteps), C.c_uint64(tag)))
        self.sizes[tag] = b.shape[0]
        if on_dev:
            self._pending[tag] = A

    def tick(self) -> dict:
        ti = AgileTickInfo()
        self._check(self._lib.agile_batch_tick(self.h, C.byref(ti)))
        if self._pending and ti.admitted:
            for tag in [t for t in self._pending if self.status(t)[0] != REQ_QUEUED]:
                del self._pending[tag]
        return {f: getattr(ti, f) for f, _ in AgileTickInfo._fields_}

    def status(self, tag: int):
        st, n = C.c_int(), C.c_int64()
        self._check(self._lib.agile_batch_status(self.h, C.c_uint64(tag), C.byref(st), C.byref(n)))
        return st.value, n.value

    def result(self, tag: int, out=None):
        """(state, steps, t) of a finished request; frees its device memory."""
        n = self.sizes[tag]
        shape = (n, 5, 16, 16, 16)
        steps, t = C.c_int64(), C.c_double()
        if out is not None and _is_device(out):
            A = _device_out(out, shape, "result")
            rc = self._lib.agile_batch_result(self.h, C.c_uint64(tag), A.data_ptr(), A.numel(), 1,
                                              C.byref(steps), C.byref(t))
        else:
            A = _host_out(out, shape, "result")
            rc = self._lib.agile_batch_result(self.h, C.c_uint64(tag), A.ctypes.data, A.size, 0, C.byref(steps),
                                              C.byref(t))
        self._check(rc)
        self.sizes.pop(tag, None)
        return A, steps.value, t.value

    def regrid(self, tag: int, refine, coarsen, max_level, variable: int = 0, eps: float = 0.01) -> dict:
        """Regrid a running request between ticks (it may go back to the
        queue when its new mesh does not fit beside the others)."""
        p = regrid_params(refine, coarsen, max_level, variable, eps)
        st = AgileRegridStats()
        rc = self._lib.agile_batch_regrid(self.h, C.c_uint64(tag), C.byref(p), C.byref(st))
        if rc != OK:
            raise AgileError(rc, self._lib.agile_batch_last_error(self.h).decode() or
                             self._lib.agile_strerror(rc).decode())
        self.sizes[tag] = int(st.new_blocks)
        return {f: getattr(st, f) for f, _ in AgileRegridStats._fields_}

    def blocks(self, tag: int) -> np.ndarray:
        """Current leaf blocks of a queued or resident request."""
        n = C.c_int64()
        cap = self.sizes.get(tag, 0)
        out = np.zeros((max(cap, 1), 4), dtype=np.int32)
        self._check(self._lib.agile_batch_blocks(self.h, C.c_uint64(tag), cap, out.ctypes.data, C.byref(n)))
        return out[:n.value]

    def cancel(self, tag: int):
        self._check(self._lib.agile_batch_cancel(self.h, C.c_uint64(tag)))
        self.sizes.pop(tag, None)
        self._pending.pop(tag, None)

    def close(self):
        if getattr(self, "h", None):
            self._lib.agile_batch_destroy(self.h)
            self.h = None
        self._pool = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
