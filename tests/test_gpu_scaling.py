"""Speedup over workers (workgroups capped by lhs_set_workers): every worker
count gives the same results, and more workers give more throughput."""
import pytest

pytestmark = pytest.mark.gpu


def test_scaling_quick():
    import torch
    assert torch.cuda.is_available()
    from paper_1004_2772_amd import scaling
    print("\n[scaling] quick", flush=True)
    res = scaling.main(["--quick", "--no-cpu"])
    pts = res["gpu"]
    assert [p["workers"] for p in pts] == [4, 256]
    # the capped BFS is exact whatever the worker count; so is the order-free
    # result of the exploration without levels (G(77,7,6,3,4,2): 1078377
    # states, the oracle's count)
    assert pts[0]["bfs_levels"] == pts[1]["bfs_levels"]
    for p in pts:
        assert p["no_levels_states"] == 1078377
    assert pts[0]["no_levels_edges"] == pts[1]["no_levels_edges"]
    # 64 times the workers: clearly faster on both explorations (the model
    # explored without levels has 15 000 open states on average, so fewer
    # workgroups have work at once)
    assert pts[1]["bfs_speedup"] > 8.0
    assert pts[1]["no_levels_speedup"] > 4.0



@pytest.fixture(scope="module")
def mid_model():
    import gen
    import oracle
    m = gen.guarded_model(4242, 6, 6, 3, 4, 3)
    return m, oracle.reach(m, cap=0)


@pytest.mark.parametrize("workers", [1, 3, 64, 0])
def test_worker_caps_do_not_change_results(mid_model, workers):
    # every exploration mode, with a captured graph keyed by the worker cap
    import paper_1004_2772_amd as lhs
    m, want = mid_model
    print(f"\n[scaling] workers={workers}: {want.total} states", flush=True)
    with lhs.Table(1 << 22, m.W) as t:
        t.set_workers(workers)
        for flags in (0, lhs.REACH_F_GRAPH, lhs.REACH_F_ASYNC):
            r = lhs.reach_explore(m, cap=0, table=t, flags=flags)
            assert (r.total, r.edges, r.deadlocks) == (want.total, want.edges, want.deadlocks), flags
            if flags != lhs.REACH_F_ASYNC:
                assert r.level_counts == want.level_counts
        capped = lhs.reach_explore(m, cap=want.total // 2, table=t, flags=lhs.REACH_F_GRAPH)
        assert capped.capped and capped.total <= want.total // 2
