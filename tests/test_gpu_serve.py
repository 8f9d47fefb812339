"""Served reachability queries (continuous batching) vs the CPU oracle and vs
exploring each model alone: results must be identical in the mix."""
import json
import os
import time

import numpy as np
import pytest

import gen
import oracle

from conftest import GOLDEN, result_fields

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
    models = gen.batch_models()
    golden = _golden_mix()
    rng = np.random.default_rng(4)
    picks = rng.integers(0, len(models), size=48)
    gaps = rng.exponential(1 / 400.0, size=len(picks))      # ~400 queries/s
    print("\n[serve] 48 queries from the mix", flush=True)
    with lhs.Server(capacity=1 << 21) as srv:
        tickets = []
        for k, gap in zip(picks, gaps):
            time.sleep(gap)
            tickets.append((int(k), srv.submit(models[k])))
        times = []
        for k, t in tickets:
            r, tm = srv.wait(t)
            g = golden[k]
            assert (r.total, r.n_levels, r.level_counts, r.edges, r.deadlocks, r.capped) == \
                (g["total"], g["n_levels"], g["level_counts"], g["edges"], g["deadlocks"], g["capped"])
            times.append(tm)
        st = srv.stats()
    assert st["completed"] == len(picks)
    # continuous batching: some queries were on the GPU at the same time
    overlaps = sum(1 for i in range(len(times)) for j in range(i + 1, len(times))
                   if times[i][1] < times[j][2] and times[j][1] < times[i][2])
    print("overlapping query pairs:", overlaps, "steps:", st["steps"], flush=True)
    assert overlaps > 0


def test_serve_equals_alone(lhs):
    rng = np.random.default_rng(8)
    models = []
    for i in range(12):
        P = int(rng.integers(2, 10))
        S = int(rng.integers(1, 6))
        m = gen.guarded_model(4400 + i, P, int(rng.integers(3, 9)), S, int(rng.integers(2, 6)), 3)
        m.cap = 40_000
        models.append(m)
    alone = [lhs.reach_explore(m, capacity=1 << 17) for m in models]
    with lhs.Server(capacity=1 << 17) as srv:
        ts = [srv.submit(m) for m in models]
        got = [srv.wait(t)[0] for t in ts]
    for m, a, g in zip(models, alone, got):
        assert result_fields(a) == result_fields(g), m.describe()
        assert result_fields(g) == result_fields(oracle.reach(m)), m.describe()


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
