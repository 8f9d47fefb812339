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


# the persistent launch (default) and host rounds of level steps
MODES = pytest.mark.parametrize("rounds", [False, True], ids=["persistent", "rounds"])


def _golden_mix():
    with open(os.path.join(GOLDEN, "batch_models.json")) as f:
        return json.load(f)["models"]


@MODES
def test_serve_mix_matches_oracle(lhs, rounds):
    """48 queries drawn from the 64-model mix arrive at about 400/s, each on a
    caller table; every result, the reachable set included, equals the
    oracle's, and queries overlap on the GPU."""
    models = gen.batch_models()
    golden = _golden_mix()
    rng = np.random.default_rng(4)
    picks = rng.integers(0, len(models), size=48)
    gaps = rng.exponential(1 / 400.0, size=len(picks))      # ~400 queries/s
    print(f"\n[serve] 48 queries from the mix, caller tables, rounds={rounds}", flush=True)
    cfg = lhs.config()
    tables = [lhs.Table(1 << 21, models[k].W, cfg) for k in picks]
    try:
        with lhs.Server(capacity=1 << 21, cfg=cfg, rounds=rounds) as srv:
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


@MODES
def test_serve_equals_alone(lhs, rounds):
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
        with lhs.Server(capacity=1 << 17, cfg=cfg, rounds=rounds) as srv:
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


@MODES
def test_serve_caller_table_rules(lhs, rounds):
    """A caller table must match the query's width and the server's line
    width, and serves one query at a time; it is free again once collected."""
    m = gen.tiny_cyclic()
    with lhs.Server(capacity=1 << 16, cfg=lhs.config(line_slots=16), rounds=rounds) as srv:
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


@MODES
def test_serve_small_budget_queues(lhs, rounds):
    # room for two 2^16-slot tables of width <= 16 at a time
    models = [gen.big_model(cap=20_000 + 1000 * i) for i in range(8)]
    budget = 2 * ((1 << 16) * (8 + 4 * 16 + 8) + 4096) + 1000
    with lhs.Server(budget_bytes=budget, capacity=1 << 16, rounds=rounds) as srv:
        ts = [srv.submit(m) for m in models]
        got = [srv.wait(t)[0] for t in ts]
        st = srv.stats()
    assert st["peak_bytes"] <= budget
    for m, g in zip(models, got):
        assert result_fields(g) == result_fields(oracle.reach(m))


@MODES
def test_serve_errors(lhs, rounds):
    with lhs.Server(budget_bytes=1 << 20, capacity=1 << 12, rounds=rounds) as srv:
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
    with lhs.Server(budget_bytes=1 << 20, capacity=1 << 16, rounds=rounds) as srv:
        with pytest.raises(lhs.LhsError) as e:
            srv.submit(gen.tiny_cyclic())                 # a 2^16-slot table never fits 1 MiB
        assert e.value.name == "LHS_EBUDGET"
    if not rounds:
        # the work queue holds a full level of each query: 2^31-slot tables
        # are for the rounds server
        with lhs.Server(capacity=1 << 31) as srv:
            with pytest.raises(lhs.LhsError) as e:
                srv.submit(gen.tiny_cyclic())
            assert e.value.name == "LHS_EINVAL"


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


def test_serve_persistent_relaunch_and_wider_query(lhs):
    """The persistent launch ends once idle and a later query starts a new
    one; a query wider than the running launch's rows waits for the next
    launch (and holds the queries behind it); every result equals the
    oracle's."""
    models = gen.batch_models()
    golden = _golden_mix()
    narrow = [k for k, m in enumerate(models) if m.W <= 8][:6]
    wide = max(range(len(models)), key=lambda k: models[k].W)
    assert models[wide].W > 8
    print(f"\n[serve] relaunch; narrow {narrow}, wide {wide}", flush=True)

    def check(k, r):
        g = golden[k]
        assert (r.total, r.n_levels, r.level_counts, r.edges, r.deadlocks, r.capped) == \
            (g["total"], g["n_levels"], g["level_counts"], g["edges"], g["deadlocks"], g["capped"]), k

    with lhs.Server(capacity=1 << 21) as srv:
        k0 = narrow[0]
        check(k0, srv.wait(srv.submit(models[k0]))[0])
        time.sleep(0.5)                                 # the launch has ended meanwhile
        l1 = srv.stats()["steps"]
        check(k0, srv.wait(srv.submit(models[k0]))[0])
        assert srv.stats()["steps"] == l1 + 1
        ks = narrow + [wide] + narrow
        ts = [(k, srv.submit(models[k])) for k in ks]
        for k, t in ts:
            check(k, srv.wait(t)[0])
        assert srv.stats()["completed"] == 2 + len(ks)


def test_serve_reused_transition_buffer(lhs):
    """A query whose transition buffer is handed on to the next query while
    the launch keeps running (large queries hold it open): workgroups that
    cached the first query's transitions in LDS must not use them for the
    second.  Both results equal the oracle's."""
    models = gen.batch_models()
    golden = _golden_mix()
    big = sorted(range(len(models)), key=lambda k: -golden[k]["total"])[:4]
    a = gen.guarded_model(7101, 5, 6, 2, 3, 3, cap=30_000)
    b = gen.guarded_model(7102, 5, 6, 2, 3, 3, cap=30_000)     # same sizes, other transitions
    wa, wb = result_fields(oracle.reach(a)), result_fields(oracle.reach(b))
    assert wa != wb
    print(f"\n[serve] transition buffer handed on; holding launch with {big}", flush=True)
    with lhs.Server(capacity=1 << 21) as srv:
        hold = [srv.submit(models[k]) for k in big]
        ra, _ = srv.wait(srv.submit(a))
        steps = srv.stats()["steps"]
        rb, _ = srv.wait(srv.submit(b))
        same_launch = srv.stats()["steps"] == steps
        for t in hold:
            srv.wait(t)
    assert result_fields(ra) == wa
    assert result_fields(rb) == wb
    print("second query in the same launch:", same_launch, flush=True)


def test_serve_query_without_lds_transitions_joins_a_launch(lhs):
    """A query posted to a running launch whose LDS holds fewer transition
    entries than it has reads its transitions from memory, and its narrower
    tile rows and masks land where the running queries' LDS copies of their
    transitions lie: those copies must be staged again, not trusted.  The
    running queries (widths 10-17, at most 96 transitions) and the joining
    ones (width 7, 228 and 288 transitions) are large, so their tiles
    interleave on the same workgroups; every result equals the oracle's."""
    models = gen.batch_models()
    golden = _golden_mix()
    hold = [58, 44, 34, 46, 14] * 2
    join = [61, 53]
    plk = lambda k: models[k].P * models[k].L * models[k].K
    assert max(plk(k) for k in hold) < min(plk(k) for k in join)
    assert min(models[k].W for k in hold) > max(models[k].W for k in join)

    def check(k, r):
        g = golden[k]
        assert (r.total, r.n_levels, r.level_counts, r.edges, r.deadlocks) == \
            (g["total"], g["n_levels"], g["level_counts"], g["edges"], g["deadlocks"]), k

    print(f"\n[serve] queries {join} posted to the launch of queries {hold}", flush=True)
    with lhs.Server(capacity=1 << 21) as srv:
        # every table allocated once and pooled, so that posting is quick
        for t in [srv.submit(models[k]) for k in hold + join]:
            srv.wait(t)
        time.sleep(0.1)                        # that launch has ended
        l0 = srv.stats()["steps"]
        th = [(k, srv.submit(models[k])) for k in hold]
        time.sleep(0.001)                      # the next launch has started
        tj = [(k, srv.submit(models[k])) for k in join]
        for k, t in th + tj:
            check(k, srv.wait(t)[0])
        launches = srv.stats()["steps"] - l0
    print("launches:", launches, flush=True)
    assert launches == 1


@MODES
def test_serve_destroy_with_queries_outstanding(lhs, rounds):
    """Destroying a server while queries are queued and on the GPU ends every
    one of them first (the worker drains its queue) and returns; a caller
    table it held is free again afterwards and keeps its query's set."""
    models = gen.batch_models()
    golden = _golden_mix()
    big = sorted(range(len(models)), key=lambda k: -golden[k]["total"])[:3]
    k0 = big[0]
    print(f"\n[serve] destroy with {big} and more outstanding, rounds={rounds}", flush=True)
    with lhs.Table(1 << 21, models[k0].W, lhs.config()) as t:
        srv = lhs.Server(capacity=1 << 21, cfg=lhs.config(), rounds=rounds)
        srv.submit(models[k0], table=t)
        for k in big[1:] + list(range(8)):
            srv.submit(models[k])
        t0 = time.time()
        srv.close()
        assert time.time() - t0 < 60
        rows, _ = t.dump()
        assert len(rows) == golden[k0]["total"]
        d = oracle.digest(rows)
        assert [d[0], hex(d[1]), hex(d[2])] == golden[k0]["digest"]
