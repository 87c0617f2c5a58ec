"""Host-side parts of the serving loop: the seeded request stream, the initial
states it asks for, and the latency percentiles (no GPU)."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2607_19277_amd import serving as S


@pytest.fixture(scope="module")
def reqs():
    return S.make_requests(n=512)


def test_stream_sizes_steps_and_mix(reqs):
    n = np.array([r.nblocks for r in reqs])
    steps = np.array([r.steps for r in reqs])
    assert n.min() >= 8 and n.max() <= 4096 * 1.1
    assert steps.min() >= 20 and steps.max() <= 200
    # log-uniform sizes: the median sits near the geometric mean of the range (~181)
    assert 100 < np.median(n) < 330
    lv = np.array([r.max_level for r in reqs])
    assert 0.3 < (lv == 2).mean() < 0.6
    gaps = np.array([r.gap for r in reqs])
    assert gaps.min() > 0 and abs(gaps.mean() - 1.0) < 0.15        # exponential(1)


def test_same_seed_same_stream():
    a, b = S.make_requests(n=40), S.make_requests(n=40)
    for x, y in zip(a, b):
        assert np.array_equal(x.blocks, y.blocks) and (x.steps, x.seed, x.gap) == (y.steps, y.seed, y.gap)


def test_meshes_are_valid_and_cover_the_box(reqs):
    agile = pytest.importorskip("paper_2607_19277_amd.agile")
    try:
        agile.lib()
    except ImportError:
        pytest.skip("library not built")
    for r in reqs[::16]:
        st = agile.plan(r.blocks, base_blocks=r.base, hi=r.hi, max_level=r.max_level)
        assert st["nblocks"] == r.nblocks
        vol = sum(8.0 ** -(l - 1) for l in r.blocks[:, 0])
        assert vol == pytest.approx(np.prod(r.base))


def test_initial_state_ranges(reqs):
    torch = pytest.importorskip("torch")
    for r in reqs[:6]:
        U = S.initial_state(r, "cpu").numpy()
        rho = U[:, 0]
        v = U[:, 1:4] / rho[:, None]
        p = (5.0 / 3.0 - 1.0) * (U[:, 4] - 0.5 * rho * (v * v).sum(axis=1))
        assert rho.min() >= 0.5 and rho.max() <= 2.0
        assert p.min() >= 0.5 - 1e-12 and p.max() <= 2.0 + 1e-12
        assert np.sqrt((v * v).sum(axis=1)).max() < 0.3


def test_weighted_percentile_matches_repetition():
    rng = np.random.default_rng(3)
    v = rng.random(50)
    w = rng.integers(0, 7, 50)
    rep = np.repeat(v, w)
    rep.sort()
    for q in (1, 50, 90, 99, 100):
        k = max(1, math.ceil(q / 100 * rep.size))
        assert S.percentile_weighted(v, w, q) == rep[k - 1]
