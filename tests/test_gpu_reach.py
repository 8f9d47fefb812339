"""GPU level-synchronous BFS vs the CPU oracle: reachable set, per-level
counts, edges and deadlocks must match exactly."""
import numpy as np
import pytest

import gen
import oracle
from oracle.closed_form import cyclic_summary

from conftest import load_golden, model_from_fixture, result_fields
from gpu_util import assert_same_set, check_table_invariants

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lhs():
    import torch
    assert torch.cuda.is_available()
    import paper_1004_2772_amd
    return paper_1004_2772_amd


def _capacity_for(states):
    # room for the kept states plus the overshoot of a discarded level
    return 1 << max(10, (2 * states + (1 << 16)).bit_length())


def _gpu(lhs, m, cap=None, capacity=None, tps=0):
    cap = m.cap if cap is None else cap
    if capacity is None:
        capacity = _capacity_for(cap if cap else 1 << 20)
    with lhs.Table(capacity, m.W) as t:
        t.set_threads_per_state(tps)
        r = lhs.reach_explore(m, cap=cap, table=t)
        rows, _ = check_table_invariants(t)
    return r, rows


def _compare(lhs, m, cap=None, capacity=None, tps=0):
    want = oracle.reach(m, cap=cap, keep_states=True)
    if capacity is None:
        capacity = _capacity_for(max(want.total, cap or 0))
    got, rows = _gpu(lhs, m, cap, capacity, tps)
    assert result_fields(got) == result_fields(want), m.describe()
    assert_same_set(rows, want.states, m.describe())
    assert oracle.digest(rows) == want.digest
    return got


def test_tiny_cyclic(lhs):
    print("\n[reach] cyclic 4x8", flush=True)
    m = gen.tiny_cyclic()
    got = _compare(lhs, m, capacity=1 << 16)
    assert result_fields(got) == cyclic_summary(4, 8)


@pytest.mark.parametrize("fx", load_golden("reach_fixtures.json")["fixtures"], ids=lambda f: f["name"])
def test_golden(lhs, fx):
    m = model_from_fixture(fx)
    for case in fx["cases"]:
        print(f"\n[reach] {fx['name']} cap={case['cap']}", flush=True)
        want = {k: case[k] for k in ("total", "level_counts", "edges", "deadlocks", "capped")}
        want["n_levels"] = len(case["level_counts"])
        got, rows = _gpu(lhs, m, cap=case["cap"], capacity=1 << 12)
        assert result_fields(got) == want
        assert_same_set(rows, oracle.reach(m, cap=case["cap"], keep_states=True).states, fx["name"])


@pytest.mark.parametrize("mode", ["on", "off", "narrow_tags"])
def test_merge_modes(lhs, mode):
    """Equal successors of one expansion pass merged before the table is
    probed (the default), not merged (one find-or-put per successor), or
    merged through one-bit hash tags (most tag matches are then other states
    and fall back to their own find-or-put): set, level counts, edges and
    deadlocks are the oracle's in every mode, and the merge counter says what
    happened."""
    code = {"on": lhs.MERGE_ON, "off": lhs.MERGE_OFF, "narrow_tags": lhs.MERGE_NARROW_TAGS}[mode]
    cases = [(gen.tiny_cyclic(), None), (gen.big_model(cap=1 << 18), 1 << 18)]
    cases += [(m, 5000) for m in _random_models(6, 91)]
    merged = {}
    for m, cap in cases:
        print(f"\n[reach] merge={mode} {m.describe()}", flush=True)
        want = oracle.reach(m, cap=cap, keep_states=True)
        with lhs.Table(_capacity_for(max(want.total, cap or 0)), m.W) as t:
            t.set_merge(code)
            t.set_counters(lhs.COUNT_MERGED)
            got = lhs.reach_explore(m, cap=cap, table=t)
            rows, _ = check_table_invariants(t)
            merged[m.name or m.seed] = (t.info()["merged"], got.edges)
        assert result_fields(got) == result_fields(want), m.describe()
        assert_same_set(rows, want.states, m.describe())
    print(f"[reach] merged/edges: {merged}", flush=True)
    big, edges = merged["big12x16"]
    if mode == "off":
        assert all(v == 0 for v, _ in merged.values())
    elif mode == "on":
        # neighbouring states' interleavings meet: a large share of a pass repeats
        assert big > edges // 10
    assert all(v < e or e == 0 for v, e in merged.values())


def _random_models(n, seed):
    rng = np.random.default_rng(seed)
    for i in range(n):
        P = int(rng.integers(1, 9))
        S = int(rng.integers(0, min(9, 33 - P)))
        L = int(rng.integers(2, 9))
        D = int(rng.integers(2, 6))
        K = int(rng.integers(1, 4))
        yield gen.guarded_model(7000 + i, P, L, S, D if S else 1, K)


def test_random_models(lhs):
    rng = np.random.default_rng(11)
    for i, m in enumerate(_random_models(40, 3)):
        tps = (0, 1, 4, 8, 16)[i % 5]
        print(f"\n[reach] {m.describe()} tps={tps}", flush=True)
        full = oracle.reach(m, cap=200_001)
        cap = 0 if not full.capped else 200_000
        _compare(lhs, m, cap=cap, tps=tps)
        if full.total > 10:
            _compare(lhs, m, cap=int(rng.integers(1, full.total)), tps=tps)


@pytest.mark.parametrize("tps", [0, 1, 4, 8, 16])
@pytest.mark.parametrize("cap", [1 << 12, 1 << 16, 1 << 19])
def test_big_model_capped(lhs, cap, tps):
    print(f"\n[reach] big model cap={cap} tps={tps}", flush=True)
    m = gen.big_model(cap=cap)
    got = _compare(lhs, m, tps=tps)
    assert got.capped


@pytest.mark.parametrize("W", [4, 7, 16, 32])
def test_width_range(lhs, W):
    print(f"\n[reach] width {W}", flush=True)
    P = min(W - 1, 12) if W > 1 else 1
    m = gen.guarded_model(31 + W, P, 6, W - P, 4, 3)
    _compare(lhs, m, cap=100_000)


def test_repeatable(lhs):
    m = gen.big_model(cap=1 << 15)
    a, _ = _gpu(lhs, m)
    b, _ = _gpu(lhs, m)
    assert result_fields(a) == result_fields(b)


@pytest.mark.parametrize("workers", [1, 3])
def test_level_spills_across_segments(lhs, workers):
    """With one or three workgroups every new state goes to their one or three
    segment cursors, so the 164 086-state level of this model overflows its
    first segment (2^20 slots / 8) into the next ones.  The next level reads
    it across segments, and the capped level after it is rolled back across
    them.  Counts and set equal the oracle's."""
    m = gen.big_model(cap=400_000)
    print(f"\n[reach] level spill, {workers} workgroup(s)", flush=True)
    want = oracle.reach(m, keep_states=True)
    assert max(want.level_counts) > (1 << 20) // 8
    with lhs.Table(1 << 20, m.W) as t:
        t.set_workers(workers)
        got = lhs.reach_explore(m, table=t)
        rows, _ = check_table_invariants(t)
    assert result_fields(got) == result_fields(want)
    assert_same_set(rows, want.states, "big model capped at 400 000")
