"""The library's host-side regrid decision (agile_regrid_decide, no GPU)
against the oracle's decision on the same block lists and estimates."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import regrid as RG
from paper_2607_19277_amd import workloads as W


def _agile():
    from paper_2607_19277_amd import agile
    agile.lib()
    return agile


def _random_mesh(rng, base, levels):
    blocks = W.uniform_blocks(base)
    for _ in range(levels - 1):
        blocks = np.array(RG.decide(blocks, rng.random(len(blocks)), base, levels, 0.7, -1.0)[0], dtype=np.int32)
    return blocks


@pytest.mark.parametrize("seed", range(8))
def test_decision_matches_the_oracle_on_random_meshes(seed):
    agile = _agile()
    rng = np.random.default_rng(100 + seed)
    base = (3, 2, 2) if seed % 2 else (2, 2, 2)
    blocks = _random_mesh(rng, base, 3)
    err = rng.random(len(blocks))
    refine, coarsen = 0.75, 0.35
    new_o, R, P = RG.decide(blocks, err, base, 3, refine, coarsen)
    new_a, st = agile.regrid_decide(blocks, err, refine, coarsen, 3, base_blocks=base, max_level=3,
                                    hi=tuple(float(b) for b in base))
    assert [tuple(r) for r in new_a.tolist()] == new_o
    assert (st["refined"], st["coarsened"], st["new_blocks"]) == (len(R), len(P), len(new_o))


def test_decision_on_the_sedov_mesh_and_rejections():
    agile = _agile()
    blocks = W.nested_blocks((8, 8, 8), 4)
    rng = np.random.default_rng(7)
    err = rng.random(len(blocks)) * 0.5
    err[:40] = 0.9
    new_o, _, _ = RG.decide(blocks, err, (8, 8, 8), 4, 0.6, 0.1)
    new_a, _ = agile.regrid_decide(blocks, err, 0.6, 0.1, 4, base_blocks=(8, 8, 8), max_level=4)
    assert [tuple(r) for r in new_a.tolist()] == new_o
    with pytest.raises(agile.AgileError):
        agile.regrid_decide(blocks, err, 0.6, 0.1, 5, base_blocks=(8, 8, 8), max_level=4)   # above the mesh's max
    with pytest.raises(agile.AgileError):
        agile.regrid_decide(blocks, err, 0.6, 0.1, 4, eps=0.0, base_blocks=(8, 8, 8), max_level=4)
