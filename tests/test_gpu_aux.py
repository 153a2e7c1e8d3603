"""Auxiliary behaviour on the GPU: the G4_LOG plan line.

A child process (so that the environment variable is read fresh) creates a
slice, installs a plan by hand and checks the lines it prints on stderr."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
from paper_2105_00027_amd import g4
cfg = g4.Config(lx=2, ly=2, nw=16, nwex=2, nq=2, q_begin=0, q_end=4, channels=1, mode=1, max_batch=8,
                prod=1, g_in=1)
h = g4.g4_init_slice(cfg)
g4.g4_set_plan(h, tile=16)
g4.g4_destroy(h)
print("child done", flush=True)
"""


def test_plan_log_lines():
    env = dict(os.environ, G4_LOG="1", PYTHONDONTWRITEBYTECODE="1")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "child done" in r.stdout
    lines = [l for l in r.stderr.splitlines() if l.startswith("g4: ")]
    assert any(l.startswith("g4: init: channels 0x1") for l in lines), r.stderr[-2000:]
    assert any(l.startswith("g4: set_plan:") and "tile 16" in l for l in lines), r.stderr[-2000:]
