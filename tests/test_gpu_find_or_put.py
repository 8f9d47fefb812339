"""Batched find-or-put on the GPU vs the sequential CPU oracle (bit-exact)."""
import numpy as np
import pytest

import gen
import oracle

from gpu_util import check_stream_batches, check_table_invariants, dev_u32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lhs():
    import torch
    assert torch.cuda.is_available()
    import paper_1004_2772_amd
    return paper_1004_2772_amd


def _run_stream(lhs, table, stream, batch):
    import torch
    n = len(stream)
    dev = dev_u32(stream)
    seen = torch.empty(n, dtype=torch.uint8, device="cuda")
    idx = torch.empty(n, dtype=torch.int32, device="cuda")
    bounds = []
    for lo in range(0, n, batch):
        hi = min(n, lo + batch)
        table.find_or_put(dev[lo:hi], seen[lo:hi], idx[lo:hi])
        bounds.append((lo, hi))
    table.check()
    return seen.cpu().numpy(), idx.cpu().numpy().view(np.uint32), bounds


TPS = [0, 1, 4, 8, 16]


@pytest.mark.parametrize("tps", TPS)
@pytest.mark.parametrize("W", [1, 2, 3, 4, 5, 8, 16, 17, 31, 32])
@pytest.mark.parametrize("batch", [257, 1000, 1 << 30])
def test_stream_parity(lhs, W, batch, tps):
    print(f"\n[fop] W={W} batch={batch} tps={tps}", flush=True)
    rows, order = gen.dup_stream(100 + W, 3000, W, 3)
    stream = gen.gather(rows, order)
    o_seen, o_id, distinct = oracle.stream(stream)
    with lhs.Table(1 << 14, W) as t:
        t.set_threads_per_state(tps)
        seen, idx, bounds = _run_stream(lhs, t, stream, batch)
        check_stream_batches(o_id, distinct, seen, idx, bounds)
        assert t.count() == distinct
        got, _ = check_table_invariants(t)
    # the stored set is the stream's distinct rows: row by row, then by digest
    want = np.unique(stream, axis=0)
    assert np.array_equal(np.unique(got, axis=0), want)
    assert oracle.digest(got) == oracle.digest(want)


@pytest.mark.parametrize("tps", TPS)
def test_small_alphabet_many_collisions(lhs, tps):
    # W=2 vectors over a 40x40 grid: heavy in-batch duplication
    print(f"\n[fop] small alphabet tps={tps}", flush=True)
    rng = np.random.default_rng(5)
    stream = rng.integers(0, 40, size=(200_000, 2)).astype(np.uint32)
    o_seen, o_id, distinct = oracle.stream(stream)
    with lhs.Table(1 << 12, 2) as t:
        t.set_threads_per_state(tps)
        seen, idx, bounds = _run_stream(lhs, t, stream, 50_000)
        check_stream_batches(o_id, distinct, seen, idx, bounds)
        check_table_invariants(t)


@pytest.mark.parametrize("tps", TPS)
def test_one_vector_many_copies(lhs, tps):
    print(f"\n[fop] 2^20 copies of one vector tps={tps}", flush=True)
    stream = np.tile(np.arange(16, dtype=np.uint32), (1 << 20, 1))
    with lhs.Table(1 << 16, 16) as t:
        t.set_threads_per_state(tps)
        seen, idx, bounds = _run_stream(lhs, t, stream, 1 << 20)
        assert int((seen == 0).sum()) == 1 and int((seen == 1).sum()) == (1 << 20) - 1
        assert len(np.unique(idx)) == 1
        assert t.count() == 1
        print("wait_hits", t.info()["wait_hits"], "cas_failures", t.info()["cas_failures"])


@pytest.mark.parametrize("tps", TPS)
def test_full_table_and_clear(lhs, tps):
    print(f"\n[fop] capacity-16 table tps={tps}", flush=True)
    rows = gen.words(77, 17 * 4).reshape(17, 4)
    with lhs.Table(16, 4) as t:
        t.set_threads_per_state(tps)
        seen, idx, _ = _run_stream(lhs, t, rows[:16], 1 << 30)
        assert np.all(seen == 0) and sorted(idx.tolist()) == list(range(16))
        seen, idx, _ = _run_stream(lhs, t, rows[:16], 1 << 30)     # all present now
        assert np.all(seen == 1)
        import torch
        dev = dev_u32(rows[16:])
        s = torch.empty(1, dtype=torch.uint8, device="cuda")
        t.find_or_put(dev, s)
        with pytest.raises(lhs.LhsError) as e:
            t.check()
        assert e.value.name == "LHS_EFULL"
        assert int(s.cpu()[0]) == 0xFF
        t.clear()
        t.check()
        assert t.count() == 0


@pytest.mark.parametrize("tps", TPS)
def test_high_fill(lhs, tps):
    # 4000 distinct vectors in 4096 slots (97.7 % fill), then every one again
    print(f"\n[fop] high fill tps={tps}", flush=True)
    rows = np.unique(gen.words(9, 4100 * 8).reshape(4100, 8), axis=0)[:4000]
    with lhs.Table(1 << 12, 8) as t:
        t.set_threads_per_state(tps)
        seen, idx, _ = _run_stream(lhs, t, rows, 1 << 30)
        assert np.all(seen == 0)
        seen2, idx2, _ = _run_stream(lhs, t, rows, 1000)
        assert np.all(seen2 == 1) and np.array_equal(idx, idx2)
        assert t.count() == 4000
        check_table_invariants(t)


@pytest.mark.parametrize("W", [4, 16, 32])
@pytest.mark.parametrize("tps", [1, 4])
def test_unaligned_input_rows(lhs, W, tps):
    """Rows handed over one word past a 16-byte boundary (a view into a larger
    buffer) take the kernel's 4-byte staging path: same results as the oracle
    and as aligned rows."""
    import torch
    print(f"\n[fop] unaligned rows W={W} tps={tps}", flush=True)
    rows, order = gen.dup_stream(300 + W, 4000, W, 2)
    stream = gen.gather(rows, order)
    o_seen, o_id, distinct = oracle.stream(stream)
    flat = torch.zeros(stream.size + 1, dtype=torch.int32, device="cuda")
    flat[1:] = dev_u32(stream).view(-1)
    dev = flat[1:].view(len(stream), W)
    assert dev.data_ptr() % 16 == 4
    n = len(stream)
    seen = torch.empty(n, dtype=torch.uint8, device="cuda")
    idx = torch.empty(n, dtype=torch.int32, device="cuda")
    with lhs.Table(1 << 14, W) as t:
        t.set_threads_per_state(tps)
        t.find_or_put(dev, seen, idx)
        t.check()
        assert t.count() == distinct
        check_stream_batches(o_id, distinct, seen.cpu().numpy(), idx.cpu().numpy().view(np.uint32), [(0, n)])
        got, _ = check_table_invariants(t)
    assert np.array_equal(np.unique(got, axis=0), np.unique(stream, axis=0))


def test_bad_threads_per_state(lhs):
    with lhs.Table(1 << 10, 4) as t:
        for bad in (2, 3, 32):
            with pytest.raises(lhs.LhsError):
                t.set_threads_per_state(bad)


def test_empty_batch(lhs):
    import torch
    with lhs.Table(1 << 10, 4) as t:
        t.find_or_put(torch.empty((0, 4), dtype=torch.int32, device="cuda"),
                      torch.empty(0, dtype=torch.uint8, device="cuda"))
        t.check()
        assert t.count() == 0


@pytest.mark.parametrize("tps", [1, 4])
def test_lines_probed_counter(lhs, tps):
    import torch
    print(f"\n[fop] lines-probed counter tps={tps}", flush=True)
    rows = np.unique(gen.words(19, 4100 * 8).reshape(4100, 8), axis=0)[:4000]
    dev = dev_u32(rows)
    seen = torch.empty(len(rows), dtype=torch.uint8, device="cuda")
    with lhs.Table(1 << 16, 8, lhs.config(8, "double", tps, tps)) as t:
        t.find_or_put(dev[:100], seen[:100])
        assert t.info()["lines_probed"] == 0            # off by default
        t.clear()
        t.set_counters(1)
        t.find_or_put(dev, seen)                        # 6 % fill: about one line each
        lines = t.info()["lines_probed"]
        assert len(rows) <= lines <= 1.05 * len(rows)
        t.find_or_put(dev, seen)                        # all seen: one line each again
        assert 2 * len(rows) <= t.info()["lines_probed"] <= 2.1 * len(rows)
    with lhs.Table(1 << 12, 8, lhs.config(8, "double", tps, tps)) as t:
        t.set_counters(1)
        t.find_or_put(dev, seen)                        # 97.7 % fill: longer probe chains
        # a simulation of random 8-slot lines under double hashing gives
        # about 1.5 lines per insert when filling to 97.7 %
        assert 1.3 * len(rows) < t.info()["lines_probed"] < 2.0 * len(rows)
        with pytest.raises(lhs.LhsError):
            t.set_counters(4)                           # bits 1 and 2 are the only counters


@pytest.mark.parametrize("tps", [0, 1])
@pytest.mark.parametrize("overlap", ["same", "windows"])
def test_concurrent_streams_one_table(lhs, tps, overlap):
    """Several calls on one table at once, each on its own stream (the table
    is lockless): every vector ends up stored once, exactly one operation
    over all calls reports it new, and every operation on it returns the
    same index."""
    import torch
    W, k_streams, n = 8, 4, 1 << 20
    rows, _ = gen.dup_stream(0xC0FFEE, n, W, 1)             # n distinct rows
    ids = []
    for k in range(k_streams):
        if overlap == "same":
            sub = np.arange(n, dtype=np.int64)               # all calls insert the same set
        else:
            sub = np.arange(k * n // 8, k * n // 8 + n // 2, dtype=np.int64)   # sliding windows
        ids.append(sub[gen.permutation(0xABC + k, len(sub)).astype(np.int64)])
    union = np.unique(np.concatenate(ids))
    print(f"\n[concurrent] {k_streams} streams, {overlap}, tps={tps}, {len(union)} distinct", flush=True)
    table = lhs.Table(1 << 22, W)
    table.set_threads_per_state(tps)
    states = [dev_u32(rows[i]) for i in ids]
    seen = [torch.empty(len(i), dtype=torch.uint8, device="cuda") for i in ids]
    idx = [torch.empty(len(i), dtype=torch.int32, device="cuda") for i in ids]
    streams = [torch.cuda.Stream() for _ in ids]
    cur = torch.cuda.current_stream()
    for s in streams:
        s.wait_stream(cur)                                   # inputs are ready
    for k, s in enumerate(streams):
        table.find_or_put(states[k], seen[k], idx[k], stream=s)
    torch.cuda.synchronize()
    table.check()
    all_ids = np.concatenate(ids)
    all_seen = np.concatenate([x.cpu().numpy() for x in seen])
    all_idx = np.concatenate([x.cpu().numpy().view(np.uint32) for x in idx])
    assert set(np.unique(all_seen).tolist()) <= {0, 1}
    info = table.info()
    # how the inserts split over the calls shows whether they overlapped
    # (run one after another, the first call would insert everything it holds)
    print(f"[concurrent] new per call {[int((x == 0).sum().item()) for x in seen]}, "
          f"waits {info['wait_hits']}, cas failures {info['cas_failures']}", flush=True)
    new_per_id = np.bincount(all_ids[all_seen == 0], minlength=n)
    assert np.all(new_per_id[union] == 1) and int(new_per_id.sum()) == len(union)
    order = np.argsort(all_ids, kind="stable")
    sid, sidx = all_ids[order], all_idx[order]
    first = np.r_[True, sid[1:] != sid[:-1]]
    ref = np.repeat(sidx[first], np.diff(np.r_[np.flatnonzero(first), len(sid)]))
    assert np.array_equal(sidx, ref), "one vector, two indices"
    assert table.count() == len(union)
    check_table_invariants(table)
    stored, sidx2 = table.dump()
    assert np.array_equal(np.sort(sidx2), np.sort(sidx[first]))
    table.close()


def test_host_buffers_refused(lhs):
    """Host memory passed for a device argument is refused by the binding
    before any kernel sees it."""
    import torch
    with lhs.Table(1 << 12, 4) as t:
        rows = torch.zeros((8, 4), dtype=torch.int32)
        seen = torch.empty(8, dtype=torch.uint8, device="cuda")
        with pytest.raises(ValueError):
            t.find_or_put(rows, seen)
        with pytest.raises(ValueError):
            t.find_or_put(rows.cuda(), torch.empty(8, dtype=torch.uint8))
        with pytest.raises(ValueError):
            t.find_or_put(rows.cuda(), seen, torch.empty(8, dtype=torch.int32))
        t.find_or_put(rows.cuda(), seen)
        t.check()
        assert sorted(seen.cpu().tolist()) == [0] + [1] * 7   # one of the equal rows inserts


@pytest.mark.parametrize("W,tps", [(1, 0), (4, 0), (4, 4)])
def test_max_capacity_2p32(lhs, W, tps):
    """The largest table the API allows, 2^32 slots (32 GiB of slots, 16 or
    64 GiB of rows): slot indices and line numbers use all 32 bits, and row
    offsets (slot x W) pass 2^32 words at W = 4.  2^21 operations (2^20 rows
    drawn twice, shuffled) in two calls, against the oracle; the stored set
    by sorted rows; each dumped row's slot is the index its find-or-put
    returned."""
    import torch
    torch.cuda.empty_cache()   # room for the table beside torch's cached blocks
    cfg = None if tps == 0 else lhs.config(16, "double", tps, tps)
    print(f"\n[fop] capacity 2^32 W={W} tps={tps}", flush=True)
    rows, order = gen.dup_stream(0x32 + W, 1 << 20, W, 2)
    stream = gen.gather(rows, order)
    o_seen, o_id, distinct = oracle.stream(stream)
    with lhs.Table(1 << 32, W, cfg) as t:
        seen, idx, bounds = _run_stream(lhs, t, stream, 1 << 20)
        check_stream_batches(o_id, distinct, seen, idx, bounds)
        assert t.count() == distinct
        got, slots = t.dump()
    # indices reach the upper half of the 32-bit range
    assert int(idx.max()) >= 1 << 31
    assert np.array_equal(np.unique(got, axis=0), np.unique(stream, axis=0))
    # the row stored in each slot is the row whose operations returned it
    pos = np.searchsorted(slots, idx)
    assert np.array_equal(slots[pos], idx)
    assert np.array_equal(got[pos], stream)
