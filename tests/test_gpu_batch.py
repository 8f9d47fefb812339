"""Batched exploration (many models in one launch) vs the CPU oracle.

Each model's result must equal the oracle's (per-level counts, edges,
deadlocks, capped flag, and the stored set row by row) and the result of
exploring it alone, for the persistent driver and the host-loop driver."""
import json
import os

import numpy as np
import pytest

import gen
import oracle

from conftest import GOLDEN, result_fields
from gpu_util import assert_same_set

pytestmark = pytest.mark.gpu

HOST_LOOP = 1


@pytest.fixture(scope="module")
def lhs():
    import torch
    assert torch.cuda.is_available()
    import paper_1004_2772_amd
    return paper_1004_2772_amd


def _mixed_models(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        P = int(rng.integers(1, 13))
        S = int(rng.integers(0, min(9, 33 - P)))
        L = int(rng.integers(2, 10))
        D = int(rng.integers(2, 8))
        K = int(rng.integers(1, 4))
        out.append(gen.guarded_model(9100 + i + 100 * seed, P, L, S, D if S else 1, K))
    return out


@pytest.mark.parametrize("flags", [0, HOST_LOOP], ids=["persistent", "host_loop"])
def test_batch_small_vs_oracle(lhs, flags):
    models = _mixed_models(24, 1)
    rng = np.random.default_rng(2)
    caps, wants = [], []
    for m in models:
        full = oracle.reach(m, cap=50_001)
        cap = 50_000 if full.capped else (int(rng.integers(1, full.total + 1)) if rng.random() < 0.3 else 0)
        caps.append(cap)
        wants.append(oracle.reach(m, cap=cap, keep_states=True))
    print(f"\n[batch] 24 mixed models flags={flags}", flush=True)
    tables = [lhs.Table(1 << 17, m.W) for m in models]
    try:
        got = lhs.reach_explore_batch(models, tables=tables, caps=caps, flags=flags)
        for m, g, w, t in zip(models, got, wants, tables):
            assert result_fields(g) == result_fields(w), m.describe()
            rows, _ = t.dump()
            assert_same_set(rows, w.states, m.describe())
            assert oracle.digest(rows) == w.digest, m.describe()
    finally:
        for t in tables:
            t.close()


@pytest.mark.parametrize("mode", ["off", "narrow_tags"])
def test_batch_merge_modes_vs_oracle(lhs, mode):
    """The persistent batch with equal successors not merged, or merged
    through one-bit tags, on half of its tables: every result is still the
    oracle's."""
    code = {"off": lhs.MERGE_OFF, "narrow_tags": lhs.MERGE_NARROW_TAGS}[mode]
    models = _mixed_models(12, 4) + [gen.big_model(cap=1 << 16)]
    caps = [40_000] * 12 + [1 << 16]
    wants = [oracle.reach(m, cap=c, keep_states=True) for m, c in zip(models, caps)]
    print(f"\n[batch] merge={mode} 13 models", flush=True)
    tables = [lhs.Table(1 << 18, m.W) for m in models]
    try:
        for i, t in enumerate(tables):
            if i % 2 == 0:
                t.set_merge(code)
        got = lhs.reach_explore_batch(models, tables=tables, caps=caps)
        for m, g, w, t in zip(models, got, wants, tables):
            assert result_fields(g) == result_fields(w), m.describe()
            rows, _ = t.dump()
            assert_same_set(rows, w.states, m.describe())
    finally:
        for t in tables:
            t.close()


def test_batch_equals_alone(lhs):
    models = _mixed_models(8, 3) + [gen.big_model(cap=1 << 16), gen.tiny_cyclic()]
    for m in models:
        m.cap = m.cap or 60_000      # keeps every model inside its 2^18-slot table
    alone = []
    for m in models:
        alone.append(lhs.reach_explore(m, capacity=1 << 18))
    print("\n[batch] batch == alone", flush=True)
    for flags in (0, HOST_LOOP):
        got = lhs.reach_explore_batch(models, capacity=1 << 18, flags=flags)
        for m, g, a in zip(models, got, alone):
            assert result_fields(g) == result_fields(a), m.describe()


def test_single_model_batch(lhs):
    m = gen.big_model(cap=1 << 18)
    want = oracle.reach(m)
    got = lhs.reach_explore_batch([m], capacity=1 << 20)[0]
    assert result_fields(got) == result_fields(want)


def test_batch_mix_64_vs_oracle(lhs):
    with open(os.path.join(GOLDEN, "batch_models.json")) as f:
        golden = json.load(f)["models"]
    models = gen.batch_models()
    assert len(models) == len(golden) == 64
    print(f"\n[batch] 64-model mix, {sum(g['total'] for g in golden)} states", flush=True)
    tables = [lhs.Table(1 << 21, m.W) for m in models]
    try:
        got = lhs.reach_explore_batch(models, tables=tables)
        print(f"batch gpu {got[0].gpu_ms:.1f} ms", flush=True)
        for m, g, want, t in zip(models, got, golden, tables):
            assert (g.total, g.n_levels, g.level_counts, g.edges, g.deadlocks, g.capped) == \
                (want["total"], want["n_levels"], want["level_counts"], want["edges"],
                 want["deadlocks"], want["capped"]), m.name
            rows, _ = t.dump()
            d = oracle.digest(rows)
            assert [d[0], hex(d[1]), hex(d[2])] == want["digest"], m.name
            # every model has at most 10^6 states: compare the sets row by row
            assert_same_set(rows, oracle.reach(m, keep_states=True).states, m.name)
    finally:
        for t in tables:
            t.close()


def test_batch_rejects_bad_input(lhs):
    with pytest.raises(lhs.LhsError):
        lhs.reach_explore_batch([], capacity=1 << 10)
    m = gen.tiny_cyclic()
    with lhs.Table(1 << 12, m.W + 1) as wrong:
        with pytest.raises(lhs.LhsError):
            lhs.reach_explore_batch([m], tables=[wrong])
