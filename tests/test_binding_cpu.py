"""Host-side checks of the boundary that need no GPU: the binding refuses
output buffers of the wrong dtype, shape or layout before any pointer crosses
the C-ABI; no C++ exception leaves an entry point (a failed host allocation
comes back as AGILE_ENOMEM); the caller-pool sizing agrees with the plan."""
from __future__ import annotations

import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

from paper_2607_19277_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _agile():
    from paper_2607_19277_amd import agile
    if not os.path.exists(agile.LIB_PATH):
        pytest.skip("libagile.so not built")
    return agile


@pytest.mark.parametrize("bad", ["float32", "shape", "strided", "readonly"])
def test_host_outputs_are_checked_before_the_call(bad):
    A = _agile()
    m = A.Mesh()            # no blocks: nothing on the device yet
    m.n = 2
    shape = (2, 5, 16, 16, 16)
    gshape = (2, 6, 5, 512)
    def make(sh):
        if bad == "float32":
            return np.empty(sh, dtype=np.float32)
        if bad == "shape":
            return np.empty((sh[0] + 1,) + sh[1:])
        if bad == "strided":
            return np.empty(sh[:-1] + (2 * sh[-1],))[..., ::2]
        a = np.empty(sh)
        a.flags.writeable = False
        return a
    with pytest.raises(ValueError):
        m.readback(make(shape))
    with pytest.raises(ValueError):
        m.read_ghosts(make(gshape))
    with pytest.raises(ValueError):
        A._host_out(make(shape), shape, "result")
    # a float32 array with twice the elements has the byte size of the float64
    # output but is still refused (the capacity is counted in doubles)
    with pytest.raises(ValueError):
        m.readback(np.empty((4, 5, 16, 16, 16), dtype=np.float32))
    m.close()


def test_config_carries_the_pool_fields():
    A = _agile()
    cfg = A.make_config()
    assert cfg.dev_pool is None and cfg.dev_pool_bytes == 0
    bc = A.AgileBatchConfig()
    assert hasattr(bc, "dev_pool") and hasattr(bc, "dev_pool_bytes")
    with pytest.raises(ValueError):
        A._pool_args(np.zeros(16))          # a host array is not a device pool


def test_plan_device_bytes_cover_the_state():
    """device_bytes is the least caller pool a mesh accepts: at least the two
    stage buffers and the x-boundary copies, and a third buffer with SSP-RK3."""
    A = _agile()
    w = W.sedov(base_blocks=4, nlevels=3)
    kw = dict(base_blocks=w.base, lo=w.lo, hi=w.hi, max_level=w.max_level)
    b2 = A.plan(w.blocks, **kw)["device_bytes"]
    b3 = A.plan(w.blocks, rk_stages=3, **kw)["device_bytes"]
    n = w.nblocks
    assert b2 >= n * (2 * 5 * 4096 + 2 * 5 * 1024) * 8
    assert b3 - b2 >= n * (5 * 4096 + 5 * 1024) * 8
    bm = A.plan(w.blocks, physics=A.MHD_GLM, riemann=A.HLL, **kw)["device_bytes"]
    assert bm >= n * (2 * 9 * 4096 + 2 * 9 * 1024) * 8   # MHD: two stage buffers and their x-boundary copies


def test_no_exception_crosses_the_abi():
    """With the address space capped just above what the process holds, the
    host tables of a 4M-block plan cannot be allocated: agile_plan returns
    AGILE_ENOMEM instead of terminating the process."""
    code = textwrap.dedent(f"""
        import ctypes as C, resource, sys
        sys.path.insert(0, {ROOT!r})
        import numpy as np
        from paper_2607_19277_amd import agile as A
        from paper_2607_19277_amd import workloads as W
        L = A.lib()
        base = (256, 128, 128)
        b = W.uniform_blocks(base)
        cfg = A.make_config(base_blocks=base, hi=(2.0, 1.0, 1.0))
        st = A.AgilePlanStats()
        msg = C.create_string_buffer(256)
        vm = [int(l.split()[1]) for l in open('/proc/self/status') if l.startswith('VmSize')][0] * 1024
        resource.setrlimit(resource.RLIMIT_AS, (vm + (96 << 20), resource.RLIM_INFINITY))
        rc = L.agile_plan(C.byref(cfg), b.shape[0], b.ctypes.data, C.byref(st), msg, 256)
        print("rc", rc, flush=True)
    """)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                       env={**os.environ, "OMP_NUM_THREADS": "1"})
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
    assert "rc -2" in r.stdout, r.stdout


def test_too_small_caller_pool_is_refused_without_touching_it():
    """A caller pool below plan()["device_bytes"] is refused with AGILE_ENOMEM
    before any device work (the pool pointer is never dereferenced, so a fake
    aligned address serves here); a misaligned pool is refused as well, and a
    pool without its size."""
    import ctypes as C
    A = _agile()
    w = W.uniform_random(nb=2, riemann=W.HLLC)
    need = A.plan(w.blocks, base_blocks=w.base, lo=w.lo, hi=w.hi)["device_bytes"]
    L = A.lib()
    for ptr, nbytes, want in ((1 << 20, need - 256, A.ENOMEM), ((1 << 20) + 64, 4 * need, A.EINVAL)):
        cfg = A.make_config(riemann=w.riemann, base_blocks=w.base, lo=w.lo, hi=w.hi)
        cfg.dev_pool, cfg.dev_pool_bytes = C.c_void_p(ptr), nbytes
        h = C.c_void_p()
        assert L.agile_mesh_create(C.byref(cfg), C.byref(h)) == A.OK
        U = np.ascontiguousarray(w.U)
        b = np.ascontiguousarray(w.blocks, dtype=np.int32)
        rc = L.agile_set_blocks(h, b.shape[0], b.ctypes.data, U.ctypes.data, 0)
        assert rc == want, (rc, L.agile_last_error(h))
        assert b"pool" in L.agile_last_error(h)
        L.agile_mesh_destroy(h)
    cfg = A.make_config(base_blocks=(1, 1, 1))
    cfg.dev_pool, cfg.dev_pool_bytes = C.c_void_p(1 << 20), 0
    h = C.c_void_p()
    assert L.agile_mesh_create(C.byref(cfg), C.byref(h)) == A.EINVAL     # a pool needs its size


def test_plan_of_32_blocks_is_the_plan_of_their_tiles():
    """A mesh of 32^3 blocks is planned as the mesh of their 16^3 tiles: the
    same tables and device bytes; a 2:1 violation between 32^3 blocks is
    refused as such."""
    A = _agile()
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from test_gpu_blocksize import to_tiles
    w = W.smooth_random(W.refine_blocks(W.uniform_blocks((2, 2, 2)), [0]), (2, 2, 2), 2, seed=11, bn=32)
    t = to_tiles(w)
    p32 = A.plan(w.blocks, base_blocks=w.base, max_level=2, block_n=32)
    p16 = A.plan(t.blocks, base_blocks=t.base, max_level=2)
    assert p32["nblocks"] == w.nblocks and p16["nblocks"] == 8 * w.nblocks
    for k in ("restrict_tasks", "prolong_tasks", "reflux_blocks", "flux_registers", "device_bytes", "levels"):
        assert p32[k] == p16[k], k
    bad = np.array([(1, 1, 0, 0), (1, 0, 1, 0), (1, 1, 1, 0)] + [(1, x, y, 1) for x in (0, 1) for y in (0, 1)] +
                   [(3, x, y, z) for x in range(4) for y in range(4) for z in range(4)], dtype=np.int32)
    with pytest.raises(A.AgileError):
        A.plan(bad, base_blocks=(2, 2, 2), max_level=3, block_n=32)
    with pytest.raises(A.AgileError):
        A.plan(w.blocks, base_blocks=w.base, max_level=2, block_n=48)


def test_stage_shape_options_before_any_block():
    """The stage-shape options are host state until blocks are set: setting
    the shape of all stages sets the last stage's too, the last stage's can
    then differ, and slab depths other than 16, 8, 4 are refused."""
    A = _agile()
    m = A.Mesh()
    assert m.get_option(A.OPT_KSLAB) == 0 and m.get_option(A.OPT_XCD) == 0   # 0: depth from the block count
    m.set_option(A.OPT_KSLAB, 8)
    m.set_option(A.OPT_XCD, 1)
    assert m.get_option(A.OPT_KSLAB_LAST) == 8 and m.get_option(A.OPT_XCD_LAST) == 1
    m.set_option(A.OPT_KSLAB_LAST, 4)
    m.set_option(A.OPT_XCD_LAST, 0)
    assert (m.get_option(A.OPT_KSLAB), m.get_option(A.OPT_XCD)) == (8, 1)
    assert (m.get_option(A.OPT_KSLAB_LAST), m.get_option(A.OPT_XCD_LAST)) == (4, 0)
    for opt in (A.OPT_KSLAB, A.OPT_KSLAB_LAST):
        with pytest.raises(A.AgileError):
            m.set_option(opt, 12)
    with pytest.raises(A.AgileError):
        m.set_option(5, 1)
    m.close()
