"""Counterexample traces (REACH_F_PARENTS): every recorded path starts at s0,
each step is a transition of the model (checked with the oracle's
next-state function), its length is the state's BFS depth + 1 (depths from
the oracle's BFS), recorded deadlock states have no successors, and the
exploration's results are unchanged by the recording."""
import numpy as np
import pytest

import gen
import oracle

from conftest import load_golden, model_from_fixture, result_fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lhs():
    import torch
    assert torch.cuda.is_available()
    import paper_1004_2772_amd
    return paper_1004_2772_amd


def _depths(m, cap):
    want = oracle.reach(m, cap=cap, keep_states=True)
    depth = {}
    at = 0
    for d, c in enumerate(want.level_counts):
        for row in want.states[at:at + c]:
            depth[row.tobytes()] = d
        at += c
    return want, depth


def _succ_set(m, row):
    return {r.tobytes() for r in oracle.successors(m, row)}


def _check_model(lhs, m, cap, flags, n_sample=200, seed=0):
    want, depth = _depths(m, cap)
    with lhs.Table(1 << 18, m.W) as t:
        got = lhs.reach_explore(m, cap=cap, table=t, flags=flags | lhs.REACH_F_PARENTS)
        assert result_fields(got) == result_fields(want), m.describe()
        rows, slots = t.dump()
        assert oracle.digest(rows) == want.digest
        rng = np.random.default_rng(seed)
        pick = rng.choice(len(slots), size=min(n_sample, len(slots)), replace=False)
        init = np.asarray(m.init, dtype=np.uint32)
        for i in pick:
            path, prow = t.trace(int(slots[i]))
            assert path[-1] == slots[i] and np.array_equal(prow[-1], rows[i])
            assert np.array_equal(prow[0], init)
            assert len(path) == depth[rows[i].tobytes()] + 1
            for a, b in zip(prow[:-1], prow[1:]):
                assert b.tobytes() in _succ_set(m, a)
        n_dead, dslots = t.deadlock_slots()
        by_slot = {int(s): r for s, r in zip(slots, rows)}
        for s in dslots:
            row = by_slot[int(s)]
            assert len(oracle.successors(m, row)) == 0
            path, prow = t.trace(int(s))
            assert len(path) == depth[row.tobytes()] + 1
        if not got.capped:
            assert n_dead == got.deadlocks
        else:
            assert n_dead >= got.deadlocks
    return got


@pytest.mark.parametrize("flags", [0, 2], ids=["host_loop", "graph"])
def test_traces_golden_fixtures(lhs, flags):
    for fx in load_golden("reach_fixtures.json")["fixtures"]:
        m = model_from_fixture(fx)
        for case in fx["cases"]:
            print(f"\n[trace] {fx['name']} cap={case['cap']}", flush=True)
            _check_model(lhs, m, case["cap"], flags)


@pytest.mark.parametrize("tps", [1, 4])
def test_traces_random_models(lhs, tps):
    rng = np.random.default_rng(41 + tps)
    for i in range(10):
        P = int(rng.integers(2, 8))
        S = int(rng.integers(1, 6))
        m = gen.guarded_model(5200 + i, P, int(rng.integers(2, 8)), S, int(rng.integers(2, 8)), 3)
        full = oracle.reach(m, cap=40_001)
        cap = 40_000 if full.capped else 0
        print(f"\n[trace] {m.describe()} cap={cap} tps={tps}", flush=True)
        _check_model(lhs, m, cap, 0, n_sample=50, seed=i)


def test_traces_big_model_capped(lhs):
    m = gen.big_model(cap=1 << 16)
    print("\n[trace] big model cap=2^16", flush=True)
    _check_model(lhs, m, 1 << 16, 0, n_sample=100)


def test_trace_rejects(lhs):
    m = gen.tiny_cyclic()                          # 4096 states
    with lhs.Table(1 << 13, m.W) as t:
        lhs.reach_explore(m, table=t)              # no records
        with pytest.raises(lhs.LhsError):
            t.trace(0)
        lhs.reach_explore(m, table=t, flags=lhs.REACH_F_PARENTS)
        slots = t.dump_slots()
        empty = int(np.flatnonzero(slots == 0)[0])
        with pytest.raises(lhs.LhsError):
            t.trace(empty)                          # no state in that slot
        t.clear()
        with pytest.raises(lhs.LhsError):
            t.trace(0)                              # records dropped by clear
