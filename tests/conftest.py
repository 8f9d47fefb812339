import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def model_from_fixture(fx):
    """gen.Model from a golden fixture entry (explicit table or cyclic)."""
    import gen
    if "cyclic" in fx:
        N, L = fx["cyclic"]
        return gen.cyclic_model(N, L)
    t = np.array(fx["trans"], dtype=np.int64)
    t[t < 0] = gen.NONE
    return gen.Model(fx["P"], fx["L"], fx["S"], fx["D"], fx["K"],
                     np.ascontiguousarray(t.astype(np.uint32)),
                     np.array(fx["init"], dtype=np.uint32), 0, fx["name"])


def result_fields(r):
    """Comparable summary of an oracle / brute / GPU result."""
    if isinstance(r, dict):
        return {k: r[k] for k in ("total", "n_levels", "level_counts", "edges", "deadlocks", "capped")}
    return dict(total=int(r.total), n_levels=int(r.n_levels),
                level_counts=[int(x) for x in r.level_counts], edges=int(r.edges),
                deadlocks=int(r.deadlocks), capped=bool(r.capped))
