"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/agile.h, and its host-side mesh planning (validation,
neighbour classification, task counts) agrees with an independent brute-force
classification written here."""
from __future__ import annotations

import os
import re

import numpy as np
import pytest

from paper_2607_19277_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "agile.h")


def _agile():
    from paper_2607_19277_amd import agile
    if not os.path.exists(agile.LIB_PATH):
        pytest.skip("libagile.so not built")
    return agile


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(agile_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_entry_point():
    agile = _agile()
    L = agile.lib()
    names = declared_functions()
    assert "agile_step" in names and "agile_set_blocks" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(agile.EXPORTS)


def test_strerror_and_bad_config():
    agile = _agile()
    L = agile.lib()
    assert L.agile_strerror(-5) == b"non-physical state"
    import ctypes as C
    cfg = agile.make_config(base_blocks=(2, 2, 2))
    cfg.block_n = 8
    h = C.c_void_p()
    assert L.agile_mesh_create(C.byref(cfg), C.byref(h)) == agile.EINVAL
    cfg = agile.make_config(base_blocks=(2, 2, 2), hi=(1.0, 2.0, 1.0))   # non-cubic cells
    assert L.agile_mesh_create(C.byref(cfg), C.byref(h)) == agile.EINVAL


def brute_classify(blocks, base):
    """For every leaf face: 'same', 'coarse' (neighbour coarser) or 'fine'."""
    leaves = {tuple(r) for r in blocks.tolist()}
    out = []
    for (l, x, y, z) in blocks.tolist():
        n = [b * 2 ** (l - 1) for b in base]
        for f in range(6):
            d, s = f // 2, f % 2
            c = [x, y, z]
            c[d] = (c[d] + (1 if s else -1)) % n[d]
            if (l, *c) in leaves:
                out.append("same")
            elif l > 1 and (l - 1, c[0] // 2, c[1] // 2, c[2] // 2) in leaves:
                out.append("coarse")
            else:
                out.append("fine")
    return out


@pytest.mark.parametrize("mesh", ["uniform", "nested3", "sedov"])
def test_plan_counts_match_brute_force(mesh):
    agile = _agile()
    if mesh == "uniform":
        blocks, base, L = W.uniform_blocks((4, 4, 4)), (4, 4, 4), 1
    elif mesh == "nested3":
        blocks, base, L = W.nested_blocks((4, 4, 4), 3), (4, 4, 4), 3
    else:
        blocks, base, L = W.nested_blocks((8, 8, 8), 4), (8, 8, 8), 4
    st = agile.plan(blocks, base_blocks=base, max_level=L)
    cls = brute_classify(blocks, base)
    assert st["nblocks"] == len(blocks)
    assert st["same_level_faces"] == cls.count("same")
    assert st["prolong_tasks"] == cls.count("coarse")
    assert st["restrict_tasks"] == cls.count("fine")
    coarse_blocks = {q for q in range(len(blocks)) if "fine" in cls[6 * q:6 * q + 6]}
    assert st["reflux_blocks"] == len(coarse_blocks)
    assert st["flux_registers"] == cls.count("coarse") + cls.count("fine")
    # correction and restriction share a launch iff no block borders both a
    # finer and a coarser block
    both = [q for q in range(len(blocks)) if "fine" in cls[6 * q:6 * q + 6] and "coarse" in cls[6 * q:6 * q + 6]]
    assert st["fused_correction"] == (0 if both else 1)
    if mesh == "sedov":
        assert (st["nblocks"], st["restrict_tasks"], st["prolong_tasks"], st["reflux_blocks"]) == (1856, 288, 1152, 288)
        assert st["prolong_launches"] == 1      # nested shells two blocks thick: no level waits for another
        assert st["fused_correction"] == 1
    assert st["device_bytes"] >= 2 * len(blocks) * 5 * 4096 * 8


def test_plan_rejects_bad_meshes():
    agile = _agile()
    base = W.uniform_blocks((2, 2, 2))
    with pytest.raises(agile.AgileError, match="duplicate"):
        agile.plan(np.concatenate([base, base[:1]]), base_blocks=(2, 2, 2))
    with pytest.raises(agile.AgileError, match="gap"):
        agile.plan(base[1:], base_blocks=(2, 2, 2))
    ref = W.refine_blocks(base, [0])
    with pytest.raises(agile.AgileError, match="overlaps"):
        agile.plan(np.concatenate([ref, base[:1]]), base_blocks=(2, 2, 2), max_level=2)
    with pytest.raises(agile.AgileError, match="level"):
        agile.plan(ref, base_blocks=(2, 2, 2), max_level=1)
    # a level-3 block next to a level-1 block violates 2:1 balance
    b4 = W.uniform_blocks((4, 4, 4))
    r2 = W.refine_blocks(b4, [0])                                # level-2 children of block 0
    lev2 = [q for q, r in enumerate(r2.tolist()) if r[0] == 2 and r[1:] == [0, 0, 0]]
    r3 = W.refine_blocks(r2, lev2)
    with pytest.raises(agile.AgileError, match="2:1"):
        agile.plan(r3, base_blocks=(4, 4, 4), max_level=3)
    with pytest.raises(agile.AgileError, match="range"):
        bad = base.copy()
        bad[0, 1] = 5
        agile.plan(bad, base_blocks=(2, 2, 2))


def test_prolongation_levels_wait_only_when_needed():
    """A level-3 slab prolonged from a level-2 block whose tangential ghost is
    itself prolonged from level 1 forces a second prolongation launch."""
    agile = _agile()
    blocks = W.dependent_levels_blocks()
    st = agile.plan(blocks, base_blocks=(4, 4, 4), max_level=3)
    assert st["levels"] == 3 and st["prolong_launches"] == 2
