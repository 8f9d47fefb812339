"""The exploration entry point that allocates nothing (reach_explore_noalloc)
against reach_explore on the same model and table shape, and against the CPU
oracle: two calls in a row, the second with a smaller model, then its size
limits and its level-array bound."""
import pytest

import gen
import oracle

from conftest import result_fields
from gpu_util import assert_same_set, check_table_invariants

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lhs():
    import torch
    assert torch.cuda.is_available()
    import paper_1004_2772_amd
    return paper_1004_2772_amd


def test_noalloc_matches_reach_explore(lhs):
    cases = [
        # 16-word model capped at 2^20 states in the largest table allowed:
        # the level that crosses the cap is expanded, then undone
        (gen.big_model(cap=1 << 20), lhs.NOALLOC_MAX_CAPACITY),
        # then a smaller one: 4 words, 4096 states, 29 levels
        (gen.tiny_cyclic(), 1 << 16),
    ]
    for m, capacity in cases:
        print(f"\n[noalloc] {m.describe()} cap={m.cap} table 2^{capacity.bit_length() - 1}", flush=True)
        want = oracle.reach(m, keep_states=True)
        with lhs.Table(capacity, m.W) as ref:
            alone = lhs.reach_explore(m, table=ref)
            ref_rows, _ = ref.dump()
        with lhs.Table(capacity, m.W) as t:
            got = lhs.reach_explore_noalloc(m, t)
            t.check()
            rows, _ = check_table_invariants(t)
        assert result_fields(got) == result_fields(alone) == result_fields(want), m.describe()
        assert_same_set(rows, ref_rows, m.describe())
        assert_same_set(rows, want.states, m.describe())


def test_noalloc_limits(lhs):
    m = gen.tiny_cyclic()
    with lhs.Table(lhs.NOALLOC_MAX_CAPACITY * 2, m.W) as big:
        with pytest.raises(lhs.LhsError) as e:
            lhs.reach_explore_noalloc(m, big)
        assert e.value.name == "LHS_EBUDGET"
    with lhs.Table(1 << 16, m.W) as t:
        with pytest.raises(lhs.LhsError) as e:
            lhs.reach_explore_noalloc(m, t, max_levels=10)     # the model has 29 levels
        assert e.value.name == "LHS_EINVAL"
        # the table is usable again at once
        r = lhs.reach_explore_noalloc(m, t)
        assert r.total == 4096 and r.n_levels == 29 and t.count() == 4096
