"""bench.py's command-line contract on the host (no GPU is touched): more
than one GPU is refused with a message, and unsupported domain sizes are
rejected before any device work."""
from __future__ import annotations

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env=dict(os.environ, HIP_VISIBLE_DEVICES=""))


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_domain_edge_must_be_a_table4_size():
    for cfg in ("kh", "paper", "srhd"):
        r = _run("--config", cfg, "--n", "100")
        assert r.returncode != 0 and "--n" in (r.stderr + r.stdout), cfg
