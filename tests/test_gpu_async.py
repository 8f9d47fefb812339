"""Exploration without level barriers (REACH_F_ASYNC) on the GPU against the
CPU oracle.  The order of expansion is free, so the result that is defined
is the one that does not depend on it: the reachable set (the table's
contents against the oracle's set digest), its size, the edges (successors
of every reachable state) and the deadlocks.  The result carries no level
counts.  With a state cap, the stored set must be a subset of the reachable
set, closed under the recorded predecessors, and at least the cap large."""
import numpy as np
import pytest

import gen
import oracle

from conftest import load_golden, model_from_fixture
from gpu_util import check_table_invariants

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lhs():
    import torch
    assert torch.cuda.is_available()
    import paper_1004_2772_amd
    return paper_1004_2772_amd


def _capacity_for(states):
    return 1 << max(10, (2 * states + 1024).bit_length())


def _set_fields(r):
    return dict(total=int(r.total), edges=int(r.edges), deadlocks=int(r.deadlocks), capped=bool(r.capped))


_WANT = {}


def _oracle_full(m, keep_states=False):
    key = (m.describe()["name"], keep_states)
    if key not in _WANT:
        _WANT[key] = oracle.reach(m, cap=0, keep_states=keep_states)
    return _WANT[key]


def _compare(lhs, m, capacity=None, cfg=None):
    want = _oracle_full(m)
    assert not want.capped
    capacity = capacity or _capacity_for(want.total)
    with lhs.Table(capacity, m.W, cfg) as t:
        got = lhs.reach_explore(m, cap=0, table=t, flags=lhs.REACH_F_ASYNC)
        assert got.n_levels == 0 and got.level_counts == []
        assert _set_fields(got) == _set_fields(want), m.describe()
        rows, _ = check_table_invariants(t)
    assert oracle.digest(rows) == want.digest
    return got


def test_tiny_cyclic(lhs):
    print("\n[async] cyclic 4x8", flush=True)
    got = _compare(lhs, gen.tiny_cyclic(), capacity=1 << 16)
    assert got.total == 4096 and got.edges == 4 * 4096 and got.deadlocks == 0


@pytest.mark.parametrize("fx", load_golden("reach_fixtures.json")["fixtures"], ids=lambda f: f["name"])
def test_golden_uncapped(lhs, fx):
    # the fixtures' uncapped cases carry the paper-independent closed values
    m = model_from_fixture(fx)
    for case in fx["cases"]:
        if case["cap"]:
            continue
        print(f"\n[async] {fx['name']}", flush=True)
        with lhs.Table(1 << 12, m.W) as t:
            got = lhs.reach_explore(m, cap=0, table=t, flags=lhs.REACH_F_ASYNC)
        assert (got.total, got.edges, got.deadlocks, got.capped) == \
            (case["total"], case["edges"], case["deadlocks"], False)


def _random_models(n, seed):
    rng = np.random.default_rng(seed)
    for i in range(n):
        P = int(rng.integers(1, 9))
        S = int(rng.integers(0, min(9, 33 - P)))
        L = int(rng.integers(2, 9))
        D = int(rng.integers(2, 6))
        K = int(rng.integers(1, 4))
        yield gen.guarded_model(9100 + i, P, L, S, D if S else 1, K)


def test_random_models(lhs):
    for m in _random_models(24, 3):
        want = oracle.reach(m, cap=0)
        if want.total > 2_000_000:
            continue
        print(f"\n[async] {m.describe()} {want.total} states", flush=True)
        _compare(lhs, m)


@pytest.mark.parametrize("ls", [8, 16, 32])
@pytest.mark.parametrize("tps", [1, 4, 8, 16])
def test_shapes(lhs, ls, tps):
    m = gen.guarded_model(79, 6, 6, 2, 3, 3)
    print(f"\n[async] line {ls} slots, {tps} lanes per state: {m.describe()}", flush=True)
    _compare(lhs, m, cfg=lhs.config(ls, "double", tps, tps))


def test_deep_chain(lhs):
    # one process walking 20000 local states: 20000 levels of one state each,
    # the shape on which level barriers cost the most
    L = 20000
    m = gen.cyclic_model(1, L)
    print(f"\n[async] chain of {L} states", flush=True)
    got = _compare(lhs, m, capacity=1 << 16)
    assert got.total == L and got.edges == L and got.deadlocks == 0


def test_wide_model(lhs):
    # many 256-entry chunks in flight, 133 BFS levels
    m = gen.guarded_model(77, 6, 6, 4, 4, 2)
    want = _oracle_full(m)
    print(f"\n[async] {m.describe()} {want.total} states", flush=True)
    assert want.total > 100_000
    _compare(lhs, m)


def test_capped_subset(lhs):
    m = gen.guarded_model(77, 6, 6, 4, 4, 2)
    want = _oracle_full(m, keep_states=True)
    full = {r.tobytes() for r in want.states}
    cap = want.total // 3
    print(f"\n[async] cap {cap} of {want.total}", flush=True)
    with lhs.Table(_capacity_for(want.total), m.W) as t:
        got = lhs.reach_explore(m, cap=cap, table=t, flags=lhs.REACH_F_ASYNC | lhs.REACH_F_PARENTS)
        assert got.capped and got.n_levels == 0
        rows, slots = check_table_invariants(t)
        assert len(rows) == got.total and got.total >= cap
        assert got.total < want.total
        assert all(r.tobytes() in full for r in rows)
        # every stored state's recorded predecessor chain reaches s0
        rng = np.random.default_rng(1)
        init = np.asarray(m.init, dtype=np.uint32)
        for i in rng.choice(len(slots), size=50, replace=False):
            path, prow = t.trace(int(slots[i]))
            assert np.array_equal(prow[0], init) and np.array_equal(prow[-1], rows[i])


def test_traces_are_paths(lhs):
    m = gen.guarded_model(5150, 5, 6, 3, 3, 2)
    want = oracle.reach(m, cap=0)
    print(f"\n[async] traces, {m.describe()} {want.total} states", flush=True)
    with lhs.Table(1 << 18, m.W) as t:
        got = lhs.reach_explore(m, cap=0, table=t, flags=lhs.REACH_F_ASYNC | lhs.REACH_F_PARENTS)
        assert _set_fields(got) == _set_fields(want)
        rows, slots = t.dump()
        init = np.asarray(m.init, dtype=np.uint32)
        rng = np.random.default_rng(2)
        for i in rng.choice(len(slots), size=min(100, len(slots)), replace=False):
            path, prow = t.trace(int(slots[i]))
            assert path[-1] == slots[i] and np.array_equal(prow[0], init)
            for a, b in zip(prow[:-1], prow[1:]):
                assert b.tobytes() in {r.tobytes() for r in oracle.successors(m, a)}
        n_dead, dslots = t.deadlock_slots()
        assert n_dead == want.deadlocks
        by_slot = {int(s): r for s, r in zip(slots, rows)}
        for s in dslots:
            assert len(oracle.successors(m, by_slot[int(s)])) == 0


def test_table_full(lhs):
    m = gen.tiny_cyclic()
    print("\n[async] 4096 states into 2048 slots", flush=True)
    with lhs.Table(1 << 11, m.W) as t:
        with pytest.raises(lhs.LhsError) as e:
            lhs.reach_explore(m, cap=0, table=t, flags=lhs.REACH_F_ASYNC)
        assert e.value.name == "LHS_EFULL"


def test_repeat_same_table(lhs):
    # the queue is reset between runs on one table; BFS and async alternate
    m = gen.guarded_model(79, 6, 6, 2, 3, 3)
    want = _oracle_full(m)
    with lhs.Table(_capacity_for(want.total), m.W) as t:
        for flags in (lhs.REACH_F_ASYNC, 0, lhs.REACH_F_ASYNC, lhs.REACH_F_ASYNC):
            got = lhs.reach_explore(m, cap=0, table=t, flags=flags)
            assert _set_fields(got) == _set_fields(want)


def _wide_enumeration_model(P=22, moving=10):
    """P * K = 66 > 64 candidate transitions per state (the expansion's LDS
    ring path): `moving` processes step through two local states, the rest
    only self-loop, every process also carries a guard that never holds, and
    process 0 copies its local state into the one shared variable."""
    NONE = 0xFFFFFFFF
    L, S, K = 2, 1, 3
    t = np.zeros((P, L, K, 5), dtype=np.uint32)
    for p in range(P):
        for l in range(L):
            t[p, l, 0] = [(l + 1) % L if p < moving else l, NONE, 0, NONE, 0]
            t[p, l, 1] = [l, 0, 7, NONE, 0]
            t[p, l, 2] = [l, NONE, 0, 0, l] if p == 0 else [l, 0, 9, NONE, 0]
    return gen.Model(P, L, S, 2, K, t, np.zeros(P + S, dtype=np.uint32), 0, f"wide-enum({P},{moving})", 0)


@pytest.mark.parametrize("tps", [1, 8])
def test_wide_enumeration(lhs, tps):
    m = _wide_enumeration_model()
    assert m.P * m.K > 64
    want = _oracle_full(m)
    print(f"\n[async] P*K = {m.P * m.K}, {want.total} states, tps={tps}", flush=True)
    assert want.total == 2 ** 10 * 2
    _compare(lhs, m, cfg=lhs.config(8, "double", tps, tps))
