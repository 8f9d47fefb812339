"""The binding in a fresh process, used the way the README shows: library
calls before any torch call of the caller's own."""
import os
import subprocess
import sys

import pytest

from conftest import ROOT

pytestmark = pytest.mark.gpu

SCRIPT = """
import paper_1004_2772_amd as lhs, gen
m = gen.tiny_cyclic()
with lhs.Table(1 << 16, m.W) as t:
    r = lhs.reach_explore(m, table=t)
    assert (r.total, r.n_levels) == (4096, 29), (r.total, r.n_levels)
    assert t.count() == 4096
print("ok")
"""


def test_library_calls_before_torch_in_a_fresh_process():
    print("\n[binding] fresh process, library first", flush=True)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", "")))
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-4000:]
