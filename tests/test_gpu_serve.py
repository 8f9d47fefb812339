"""Served reachability queries (continuous batching) vs the CPU oracle and vs
exploring each model alone: results must be identical in the mix, including
the reachable set, which queries run on caller tables keep."""
import json
import os
import time

import numpy as np
import pytest

import gen
import oracle

from conftest import GOLDEN, result_fields
from gpu_util import assert_same_set

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lhs():
    import torch
    assert torch.cuda.is_available()
    import paper_1004_2772_amd
    return paper_1004_2772_amd


def _golden_mix():
    with open(os.path.join(GOLDEN, "batch_models.json")) as f:
        return json.load(f)["models"]


def test_serve_mix_matches_oracle(lhs):
    """48 queries drawn from the 64-model mix arrive at about 400/s, each on a
    caller table; every result, the reachable set included, equals the
    oracle's, and queries overlap on the GPU."""
    models = gen.batch_models()
    golden = _golden_mix()
    rng = np.random.default_rng(4)
    picks = rng.integers(0, len(models), size=48)
    gaps = rng.exponential(1 / 400.0, size=len(picks))      # ~400 queries/s
    print("\n[serve] 48 queries from the mix, caller tables", flush=True)
    cfg = lhs.config()
    tables = [lhs.Table(1 << 21, models[k].W, cfg) for k in picks]
    try:
        with lhs.Server(capacity=1 << 21, cfg=cfg) as srv:
            tickets = []
            for k, gap, t in zip(picks, gaps, tables):
                time.sleep(gap)
                tickets.append((int(k), srv.submit(models[k], table=t)))
            times = []
            for k, t in tickets:
                r, tm = srv.wait(t)
                g = golden[k]
                assert (r.total, r.n_levels, r.level_counts, r.edges, r.deadlocks, r.capped) == \
                    (g["total"], g["n_levels"], g["level_counts"], g["edges"], g["deadlocks"], g["capped"])
                times.append(tm)
            st = srv.stats()
        assert st["completed"] == len(picks)
        print("comparing served sets with the oracle", flush=True)
        want = {}
        for k, t in zip(picks, tables):
            k = int(k)
            if k not in want:
                want[k] = oracle.reach(models[k], keep_states=True).states
            rows, _ = t.dump()
            assert_same_set(rows, want[k], models[k].name)
            d = oracle.digest(rows)
            assert [d[0], hex(d[1]), hex(d[2])] == golden[k]["digest"], models[k].name
    finally:
        for t in tables:
            t.close()
    # continuous batching: some queries were on the GPU at the same time
    overlaps = sum(1 for i in range(len(times)) for j in range(i + 1, len(times))
                   if times[i][1] < times[j][2] and times[j][1] < times[i][2])
    print("overlapping query pairs:", overlaps, "steps:", st["steps"], flush=True)
    assert overlaps > 0


def test_serve_equals_alone(lhs):
    """Capped and uncapped queries, all submitted at once: each served result
    and set equals the model explored alone (reach_explore on its own table)
    and the oracle's; a capped query's table holds only the kept levels."""
    rng = np.random.default_rng(8)
    models = []
    for i in range(12):
        P = int(rng.integers(2, 10))
        S = int(rng.integers(1, 6))
        m = gen.guarded_model(4400 + i, P, int(rng.integers(3, 9)), S, int(rng.integers(2, 6)), 3)
        m.cap = 40_000
        models.append(m)
    cfg = lhs.config()
    alone, alone_rows = [], []
    for m in models:
        with lhs.Table(1 << 17, m.W, cfg) as t:
            alone.append(lhs.reach_explore(m, table=t))
            alone_rows.append(t.dump()[0])
    tables = [lhs.Table(1 << 17, m.W, cfg) for m in models]
    try:
        with lhs.Server(capacity=1 << 17, cfg=cfg) as srv:
            ts = [srv.submit(m, table=t) for m, t in zip(models, tables)]
            got = [srv.wait(t)[0] for t in ts]
        n_capped = 0
        for m, a, g, t, ar in zip(models, alone, got, tables, alone_rows):
            assert result_fields(a) == result_fields(g), m.describe()
            w = oracle.reach(m, keep_states=True)
            assert result_fields(g) == result_fields(w), m.describe()
            rows, _ = t.dump()
            assert_same_set(rows, w.states, m.describe())
            assert_same_set(rows, ar, m.describe())
            n_capped += g.capped
        assert n_capped >= 3      # the discarded level of a capped query is undone
    finally:
        for t in tables:
            t.close()


def test_serve_caller_table_rules(lhs):
    """A caller table must match the query's width and the server's line
    width, and serves one query at a time; it is free again once collected."""
    m = gen.tiny_cyclic()
    with lhs.Server(capacity=1 << 16, cfg=lhs.config(line_slots=16)) as srv:
        with lhs.Table(1 << 16, m.W + 1, lhs.config(line_slots=16)) as wide, \
                lhs.Table(1 << 16, m.W, lhs.config(line_slots=8)) as narrow, \
                lhs.Table(1 << 16, m.W, lhs.config(line_slots=16)) as ok:
            for bad in (wide, narrow):
                with pytest.raises(lhs.LhsError) as e:
                    srv.submit(m, table=bad)
                assert e.value.name == "LHS_EINVAL"
            t1 = srv.submit(m, table=ok)
            with pytest.raises(lhs.LhsError) as e:
                srv.submit(m, table=ok)                 # still serving t1
            assert e.value.name == "LHS_EINVAL"
            r1, _ = srv.wait(t1)
            assert r1.total == 4096 and ok.count() == 4096
            t2 = srv.submit(gen.cyclic_model(4, 3), table=ok)
            r2, _ = srv.wait(t2)
            assert r2.total == 81 and ok.count() == 81   # cleared at admission
            with pytest.raises(lhs.LhsError) as e:
                srv.submit(m, cap=1 << 16, table=ok)   # state_cap >= capacity
            assert e.value.name == "LHS_EINVAL"


def test_serve_small_budget_queues(lhs):
    # room for two 2^16-slot tables of width <= 16 at a time
    models = [gen.big_model(cap=20_000 + 1000 * i) for i in range(8)]
    budget = 2 * ((1 << 16) * (8 + 4 * 16 + 8) + 4096) + 1000
    with lhs.Server(budget_bytes=budget, capacity=1 << 16) as srv:
        ts = [srv.submit(m) for m in models]
        got = [srv.wait(t)[0] for t in ts]
        st = srv.stats()
    assert st["peak_bytes"] <= budget
    for m, g in zip(models, got):
        assert result_fields(g) == result_fields(oracle.reach(m))


def test_serve_errors(lhs):
    with lhs.Server(budget_bytes=1 << 20, capacity=1 << 12) as srv:
        big = gen.guarded_model(5, 4, 8, 2, 3, 3)
        with pytest.raises(lhs.LhsError) as e:
            lhs.Server(capacity=24)
        assert e.value.name == "LHS_EINVAL"
        # a query that overflows its table fails alone; the next one is fine
        bad = srv.submit(gen.cyclic_model(3, 20))         # 8000 states in 4096 slots
        good = srv.submit(gen.cyclic_model(2, 8))
        with pytest.raises(lhs.LhsError) as e:
            srv.wait(bad)
        assert e.value.name == "LHS_EFULL"
        r, _ = srv.wait(good)
        assert r.total == 64
        with pytest.raises(lhs.LhsError) as e:
            srv.poll(good)
        assert e.value.name == "LHS_ENOTFOUND"
        del big
    with lhs.Server(budget_bytes=1 << 20, capacity=1 << 16) as srv:
        with pytest.raises(lhs.LhsError) as e:
            srv.submit(gen.tiny_cyclic())                 # a 2^16-slot table never fits 1 MiB
        assert e.value.name == "LHS_EBUDGET"


def test_serve_client_threads(lhs):
    """Queries submitted and awaited from several host threads at once; two
    threads waiting on one ticket: one gets the result, the other
    LHS_ENOTFOUND (the ticket is collected once)."""
    import threading
    models = gen.batch_models()
    golden = _golden_mix()
    rng = np.random.default_rng(12)
    picks = [rng.integers(0, len(models), size=6) for _ in range(4)]
    print("\n[serve] 4 client threads x 6 queries", flush=True)
    errors = []

    def fields(r):
        return (r.total, r.n_levels, r.level_counts, r.edges, r.deadlocks, r.capped)

    def gfields(g):
        return (g["total"], g["n_levels"], g["level_counts"], g["edges"], g["deadlocks"], g["capped"])

    with lhs.Server(capacity=1 << 21) as srv:
        def client(ks):
            try:
                ts = [(int(k), srv.submit(models[int(k)])) for k in ks]
                for k, t in ts:
                    if fields(srv.wait(t)[0]) != gfields(golden[k]):
                        errors.append(k)
            except Exception as e:          # reported below, on the main thread
                errors.append(repr(e))

        th = [threading.Thread(target=client, args=(ks,)) for ks in picks]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=120)
        assert not any(t.is_alive() for t in th)
        assert not errors, errors
        ticket = srv.submit(models[3])
        out = []

        def waiter():
            try:
                out.append(fields(srv.wait(ticket)[0]) == gfields(golden[3]))
            except lhs.LhsError as e:
                out.append(e.name)

        ws = [threading.Thread(target=waiter) for _ in range(2)]
        for t in ws:
            t.start()
        for t in ws:
            t.join(timeout=60)
        assert not any(t.is_alive() for t in ws)
        assert sorted(map(str, out)) == ["LHS_ENOTFOUND", "True"]
        assert srv.stats()["completed"] == 4 * 6 + 1
