"""Every table shape (line width 8/16/32 slots x probe sequence x lanes per
state) gives the oracle's results: find-or-put streams, full tables (each
probe sequence reaches every line), BFS, batches and the server.  Tables
with a tuned shape (tuning file loaded) likewise."""
import json

import numpy as np
import pytest

import gen
import oracle

from conftest import load_golden, model_from_fixture, result_fields
from gpu_util import check_stream_batches, check_table_invariants, dev_u32

pytestmark = pytest.mark.gpu

LINES = [8, 16, 32]
PROBES = ["double", "linear", "quadratic"]
SHAPES = [(ls, p) for ls in LINES for p in PROBES]


@pytest.fixture(scope="module")
def lhs():
    import torch
    assert torch.cuda.is_available()
    import paper_1004_2772_amd
    return paper_1004_2772_amd


def _stream(lhs, t, stream, batch):
    import torch
    n = len(stream)
    dev = dev_u32(stream)
    seen = torch.empty(n, dtype=torch.uint8, device="cuda")
    idx = torch.empty(n, dtype=torch.int32, device="cuda")
    bounds = []
    for lo in range(0, n, batch):
        hi = min(n, lo + batch)
        t.find_or_put(dev[lo:hi], seen[lo:hi], idx[lo:hi])
        bounds.append((lo, hi))
    t.check()
    return seen.cpu().numpy(), idx.cpu().numpy().view(np.uint32), bounds


@pytest.mark.parametrize("tps", [1, 4, 8, 16])
@pytest.mark.parametrize("ls,probe", SHAPES)
@pytest.mark.parametrize("W", [3, 16, 32])
def test_stream_shapes(lhs, ls, probe, tps, W):
    print(f"\n[shape] stream W={W} ls={ls} probe={probe} tps={tps}", flush=True)
    rows, order = gen.dup_stream(300 + W, 3000, W, 3)
    stream = gen.gather(rows, order)
    _, o_id, distinct = oracle.stream(stream)
    with lhs.Table(1 << 13, W, lhs.config(ls, probe, tps, tps)) as t:
        assert t.config() == {"line_slots": ls, "probe": probe, "tps_find_or_put": tps, "tps_expand": tps}
        seen, idx, bounds = _stream(lhs, t, stream, 1000)
        check_stream_batches(o_id, distinct, seen, idx, bounds)
        assert t.count() == distinct
        got, _ = check_table_invariants(t)
    assert oracle.digest(got) == oracle.digest(np.unique(stream, axis=0))


@pytest.mark.parametrize("tps", [1, 4, 16])
@pytest.mark.parametrize("ls,probe", SHAPES)
def test_full_table_shapes(lhs, ls, probe, tps):
    # 64 slots = 8, 4 or 2 lines: filling every slot needs a probe sequence
    # that reaches every line; the 65th vector then fails with EFULL
    import torch
    print(f"\n[shape] full 64-slot table ls={ls} probe={probe} tps={tps}", flush=True)
    rows = np.unique(gen.words(55, 80 * 4).reshape(80, 4), axis=0)[:65]
    with lhs.Table(64, 4, lhs.config(ls, probe, tps, tps)) as t:
        seen, idx, _ = _stream(lhs, t, rows[:64], 1 << 30)
        assert np.all(seen == 0) and sorted(idx.tolist()) == list(range(64))
        seen, idx2, _ = _stream(lhs, t, rows[:64], 7)
        assert np.all(seen == 1) and np.array_equal(idx, idx2)
        check_table_invariants(t)
        s = torch.empty(1, dtype=torch.uint8, device="cuda")
        t.find_or_put(dev_u32(rows[64:]), s)
        with pytest.raises(lhs.LhsError) as e:
            t.check()
        assert e.value.name == "LHS_EFULL"


@pytest.mark.parametrize("tps", [1, 4])
@pytest.mark.parametrize("ls,probe", SHAPES)
def test_high_fill_shapes(lhs, ls, probe, tps):
    print(f"\n[shape] 97.7% fill ls={ls} probe={probe} tps={tps}", flush=True)
    rows = np.unique(gen.words(9, 4100 * 8).reshape(4100, 8), axis=0)[:4000]
    with lhs.Table(1 << 12, 8, lhs.config(ls, probe, tps, tps)) as t:
        seen, idx, _ = _stream(lhs, t, rows, 1 << 30)
        assert np.all(seen == 0)
        seen2, idx2, _ = _stream(lhs, t, rows, 1000)
        assert np.all(seen2 == 1) and np.array_equal(idx, idx2)
        check_table_invariants(t)


def _bfs_models():
    yield "cyclic4x8", gen.tiny_cyclic(), 0
    fx = {f["name"]: f for f in load_golden("reach_fixtures.json")["fixtures"]}
    for name in list(fx)[:3]:
        yield name, model_from_fixture(fx[name]), 0
    yield "guarded6x8", gen.guarded_model(4242, 6, 8, 4, 4, 3), 20_000


@pytest.mark.parametrize("tps", [1, 4, 16])
@pytest.mark.parametrize("ls,probe", SHAPES)
def test_bfs_shapes(lhs, ls, probe, tps):
    for name, m, cap in _bfs_models():
        print(f"\n[shape] bfs {name} cap={cap} ls={ls} probe={probe} tps={tps}", flush=True)
        want = oracle.reach(m, cap=cap)
        with lhs.Table(1 << 17, m.W, lhs.config(ls, probe, tps, tps)) as t:
            got = lhs.reach_explore(m, cap=cap, table=t)
            rows, _ = check_table_invariants(t)
        assert result_fields(got) == result_fields(want), name
        assert oracle.digest(rows) == want.digest, name


def _batch_models():
    rng = np.random.default_rng(8)
    out = []
    for i in range(12):
        P = int(rng.integers(2, 8))
        S = int(rng.integers(1, 6))
        out.append(gen.guarded_model(9100 + i, P, int(rng.integers(3, 9)), S, int(rng.integers(2, 6)), 3))
    return out


@pytest.mark.parametrize("flags", [0, 1], ids=["persistent", "host_loop"])
@pytest.mark.parametrize("ls,probe,tps", [(8, "linear", 1), (32, "quadratic", 4), (16, "double", 16),
                                          (32, "double", 1), (8, "quadratic", 8)])
def test_batch_shapes(lhs, ls, probe, tps, flags):
    models = _batch_models()
    wants = [oracle.reach(m, cap=30_000) for m in models]
    print(f"\n[shape] batch of {len(models)} ls={ls} probe={probe} tps={tps} flags={flags}", flush=True)
    tables = [lhs.Table(1 << 17, m.W, lhs.config(ls, probe, tps, tps)) for m in models]
    try:
        got = lhs.reach_explore_batch(models, tables=tables, caps=[30_000] * len(models), flags=flags)
        for m, g, w, t in zip(models, got, wants, tables):
            assert result_fields(g) == result_fields(w), m.describe()
            rows, _ = check_table_invariants(t)
            assert oracle.digest(rows) == w.digest
    finally:
        for t in tables:
            t.close()


def test_batch_rejects_mixed_line_widths(lhs):
    models = _batch_models()[:2]
    tables = [lhs.Table(1 << 12, models[0].W, lhs.config(8)), lhs.Table(1 << 12, models[1].W, lhs.config(16))]
    try:
        with pytest.raises(lhs.LhsError) as e:
            lhs.reach_explore_batch(models, tables=tables)
        assert e.value.name == "LHS_EINVAL"
    finally:
        for t in tables:
            t.close()


@pytest.mark.parametrize("ls,probe,tps", [(8, "quadratic", 4), (32, "linear", 1)])
def test_server_shapes(lhs, ls, probe, tps):
    models = _batch_models()[:8]
    wants = [oracle.reach(m, cap=30_000) for m in models]
    print(f"\n[shape] server ls={ls} probe={probe} tps={tps}", flush=True)
    with lhs.Server(capacity=1 << 17, cfg=lhs.config(ls, probe, tps, tps)) as srv:
        tickets = [srv.submit(m, cap=30_000) for m in models]
        for m, tk, w in zip(models, tickets, wants):
            r, _ = srv.wait(tk)
            assert result_fields(r) == result_fields(w), m.describe()


def test_tuned_shapes_are_used(lhs, tmp_path):
    """A loaded tuning file decides the shape of lhs_create tables, of
    reach_explore's and the batch's internal tables; results stay exact."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    doc = {"format": "lhs-tune-1", "device": arch, "entries": [
        {"kind": "table", "W": 32, "log2_capacity": 17, "line_slots": 8, "probe": "quadratic",
         "tps_find_or_put": 8, "tps_expand": 4},
        {"kind": "batch", "W": 32, "log2_capacity": 21, "line_slots": 32, "probe": "linear",
         "tps_find_or_put": 0, "tps_expand": 16}]}
    p = tmp_path / "tune.json"
    p.write_text(json.dumps(doc))
    assert lhs.tune_load(str(p)) == 2
    try:
        with lhs.Table(1 << 17, 5) as t:
            assert t.config() == {"line_slots": 8, "probe": "quadratic", "tps_find_or_put": 8,
                                  "tps_expand": 4}
        m = gen.guarded_model(4242, 6, 8, 4, 4, 3)
        want = oracle.reach(m, cap=20_000)
        got = lhs.reach_explore(m, cap=20_000)
        assert result_fields(got) == result_fields(want)
        models = _batch_models()
        wants = [oracle.reach(mm, cap=30_000) for mm in models]
        got = lhs.reach_explore_batch(models, caps=[30_000] * len(models))
        for g, w in zip(got, wants):
            assert result_fields(g) == result_fields(w)
    finally:
        lhs.tune_clear()
