"""BFS with the level loop replayed from a captured HIP graph
(REACH_F_GRAPH) vs the CPU oracle, and vs the host-driven loop: the same
reachable set, per-level counts, edges, deadlocks and cap outcome."""
import numpy as np
import pytest

import gen
import oracle
from oracle.closed_form import cyclic_summary

from conftest import load_golden, model_from_fixture, result_fields
from gpu_util import check_table_invariants

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lhs():
    import torch
    assert torch.cuda.is_available()
    import paper_1004_2772_amd
    return paper_1004_2772_amd


def _graph(lhs, t, m, cap, max_levels=0):
    return lhs.reach_explore(m, cap=cap, table=t, flags=lhs.REACH_F_GRAPH, max_levels=max_levels)


def _check(lhs, t, m, cap):
    want = oracle.reach(m, cap=cap)
    got = _graph(lhs, t, m, cap)
    assert result_fields(got) == result_fields(want), m.describe()
    rows, _ = check_table_invariants(t)
    assert oracle.digest(rows) == want.digest
    return got


def test_graph_cyclic(lhs):
    print("\n[graph] cyclic 4x8 (29 levels: several replays)", flush=True)
    m = gen.tiny_cyclic()
    with lhs.Table(1 << 16, m.W) as t:
        got = _check(lhs, t, m, 0)
    assert result_fields(got) == cyclic_summary(4, 8)


def test_graph_golden_one_table(lhs):
    """Every golden fixture and cap on one table: the captured graph is
    reused across models of the same width and rebuilt when the transition
    layout changes."""
    fx = load_golden("reach_fixtures.json")["fixtures"]
    by_w = {}
    for f in fx:
        by_w.setdefault(model_from_fixture(f).W, []).append(f)
    for W, group in by_w.items():
        with lhs.Table(1 << 12, W) as t:
            for f in group:
                m = model_from_fixture(f)
                for case in f["cases"]:
                    print(f"\n[graph] {f['name']} cap={case['cap']}", flush=True)
                    got = _graph(lhs, t, m, case["cap"])
                    want = {k: case[k] for k in ("total", "level_counts", "edges", "deadlocks", "capped")}
                    want["n_levels"] = len(case["level_counts"])
                    assert result_fields(got) == want


@pytest.mark.parametrize("tps", [1, 4, 16])
def test_graph_random_models(lhs, tps):
    rng = np.random.default_rng(21 + tps)
    for i in range(12):
        P = int(rng.integers(1, 9))
        S = int(rng.integers(0, min(9, 33 - P)))
        m = gen.guarded_model(8100 + i, P, int(rng.integers(2, 9)), S, int(rng.integers(2, 6)) if S else 1,
                              int(rng.integers(1, 4)))
        full = oracle.reach(m, cap=100_001)
        cap = 100_000 if full.capped else 0
        print(f"\n[graph] {m.describe()} cap={cap} tps={tps}", flush=True)
        with lhs.Table(1 << 18, m.W) as t:
            t.set_threads_per_state(tps)
            _check(lhs, t, m, cap)
            if full.total > 10:
                _check(lhs, t, m, int(rng.integers(1, min(full.total, 100_000))))


@pytest.mark.parametrize("cap", [1 << 12, 1 << 19])
def test_graph_big_model_capped(lhs, cap):
    print(f"\n[graph] big model cap={cap}", flush=True)
    m = gen.big_model(cap=cap)
    with lhs.Table(1 << 21, m.W) as t:
        got = _check(lhs, t, m, cap)
        host = lhs.reach_explore(m, cap=cap, table=t)
    assert got.capped and result_fields(got) == result_fields(host)


def test_graph_max_levels(lhs):
    # 29 levels do not fit a bound of 20: the same error as the host loop
    m = gen.tiny_cyclic()
    with lhs.Table(1 << 16, m.W) as t:
        for flags in (0, lhs.REACH_F_GRAPH):
            with pytest.raises(lhs.LhsError) as e:
                lhs.reach_explore(m, table=t, flags=flags, max_levels=20)
            assert e.value.name == "LHS_EINVAL"
        got = _graph(lhs, t, m, 0, max_levels=29)
        assert got.n_levels == 29


def test_graph_internal_table(lhs):
    m = gen.guarded_model(4242, 6, 8, 4, 4, 3)
    want = oracle.reach(m, cap=20_000)
    got = lhs.reach_explore(m, cap=20_000, flags=lhs.REACH_F_GRAPH)
    assert result_fields(got) == result_fields(want)
