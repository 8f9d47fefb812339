"""The multi-core CPU lockless table (the paper's method on host cores, a
baseline next to the GPU) against the sequential oracle: streams (one new
per distinct vector, equal indices for equal vectors) and BFS (level counts,
edges, deadlocks, cap outcome and the stored set) for 1 to 8 threads."""
import numpy as np
import pytest

import cpu_table
import gen
import oracle
from oracle.closed_form import cyclic_summary

from conftest import load_golden, model_from_fixture, result_fields


@pytest.mark.parametrize("threads", [1, 4, 8])
@pytest.mark.parametrize("W", [1, 3, 16, 32])
def test_stream(W, threads):
    rows, order = gen.dup_stream(50 + W, 20_000, W, 3)
    stream = gen.gather(rows, order)
    _, o_id, distinct = oracle.stream(stream)
    seen, index, _ = cpu_table.stream(stream, 17, threads)
    assert set(np.unique(seen).tolist()) <= {0, 1}
    assert np.array_equal(np.bincount(o_id[seen == 0], minlength=distinct), np.ones(distinct))
    _, first = np.unique(o_id, return_index=True)
    assert np.array_equal(index, index[first][o_id])
    assert len(np.unique(index[first])) == distinct


def test_stream_full_table():
    rows = np.unique(gen.words(3, 20 * 4).reshape(20, 4), axis=0)[:17]
    with pytest.raises(RuntimeError):
        cpu_table.stream(rows, 4, 2)          # 16 slots, 17 distinct vectors


def _check(m, cap, threads, log2cap=18):
    want = oracle.reach(m, cap=cap)
    got = cpu_table.reach(m, cap, log2cap, threads, keep_rows=True)
    assert result_fields(got) == result_fields(want), (m.describe(), threads)
    assert oracle.digest(got.rows) == want.digest
    return got


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_cyclic(threads):
    got = _check(gen.tiny_cyclic(), 0, threads)
    assert result_fields(got) == cyclic_summary(4, 8)


def test_golden():
    for fx in load_golden("reach_fixtures.json")["fixtures"]:
        m = model_from_fixture(fx)
        for case in fx["cases"]:
            got = cpu_table.reach(m, case["cap"], 12, 4)
            want = {k: case[k] for k in ("total", "level_counts", "edges", "deadlocks", "capped")}
            want["n_levels"] = len(case["level_counts"])
            assert result_fields(got) == want, fx["name"]


@pytest.mark.parametrize("threads", [2, 8])
def test_random_models(threads):
    rng = np.random.default_rng(5 + threads)
    for i in range(15):
        P = int(rng.integers(1, 9))
        S = int(rng.integers(0, min(9, 33 - P)))
        m = gen.guarded_model(6100 + i, P, int(rng.integers(2, 9)), S, int(rng.integers(2, 6)) if S else 1,
                              int(rng.integers(1, 4)))
        full = oracle.reach(m, cap=50_001)
        _check(m, 50_000 if full.capped else 0, threads)
        if full.total > 10:
            _check(m, int(rng.integers(1, min(full.total, 50_000))), threads)
