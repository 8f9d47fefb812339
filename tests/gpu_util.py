"""Helpers for the GPU parity tests (host side only)."""
import numpy as np

MASK64 = (1 << 64) - 1
OCC = np.uint64(1 << 63)
DONE = np.uint64(1 << 62)
MEMO = np.uint64((1 << 62) - 1)


def sorted_rows(a: np.ndarray) -> np.ndarray:
    """Rows of a [n, W] uint32 array in one fixed total order (bytewise, via
    a void view): two arrays hold the same multiset of rows iff their sorted
    forms are equal."""
    a = np.ascontiguousarray(a, dtype=np.uint32)
    if a.ndim != 2 or len(a) == 0:
        return a
    v = a.view(np.dtype((np.void, a.shape[1] * 4))).ravel()
    return a[np.argsort(v, kind="stable")]


def assert_same_set(got: np.ndarray, want: np.ndarray, what=""):
    """The GPU's stored rows equal the oracle's states, row by row."""
    got = np.asarray(got, dtype=np.uint32)
    want = np.asarray(want, dtype=np.uint32)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    assert np.array_equal(sorted_rows(got), sorted_rows(want)), f"stored set differs: {what}"


def dev_u32(a):
    """numpy uint32 array -> contiguous int32 CUDA tensor with the same bits."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def _rotl(x, r):
    return (x << np.uint64(r)) | (x >> np.uint64(64 - r))


def table_hash(rows: np.ndarray, seed: int) -> np.ndarray:
    """The table's 64-bit vector hash, re-implemented on the host from its
    definition (MurmurHash3 x64 block mixing over 64-bit word pairs, the
    length xor, fmix64).  Used only to check slot invariants."""
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    n, W = rows.shape
    c1, c2 = np.uint64(0x87c37b91114253d5), np.uint64(0x4cf5ad432745937f)
    with np.errstate(over="ignore"):
        h = np.full(n, seed, dtype=np.uint64)
        i = 0
        while i + 1 < W:
            k = rows[:, i].astype(np.uint64) | (rows[:, i + 1].astype(np.uint64) << np.uint64(32))
            k = _rotl(k * c1, 31) * c2
            h = _rotl(h ^ k, 27) * np.uint64(5) + np.uint64(0x52dce729)
            i += 2
        if i < W:
            k = rows[:, i].astype(np.uint64)
            h ^= _rotl(k * c1, 31) * c2
        h ^= np.uint64(W * 4)
        h ^= h >> np.uint64(33)
        h *= np.uint64(0xff51afd7ed558ccd)
        h ^= h >> np.uint64(33)
        h *= np.uint64(0xc4ceb9fe1a85ec53)
        h ^= h >> np.uint64(33)
    return h


def check_table_invariants(table, sample=None, seed=0):
    """Invariants of a table between calls (figure of bucket states and the
    probe sequence): every non-empty slot is done; each slot's memo is its
    row's hash; every slot in front of a stored row on that row's probe
    sequence is non-empty (otherwise a later lookup would insert it again);
    no vector is stored twice.  With `sample`, the per-row checks run on that
    many random stored rows (uniqueness is then left to the caller)."""
    info = table.info()
    slots = table.dump_slots()
    all_rows, all_idx = table.dump()
    nonempty = slots != 0
    assert np.all((slots[nonempty] & (OCC | DONE)) == (OCC | DONE)), "claimed slot not done"
    assert int(nonempty.sum()) == len(all_idx)
    rows, idx = all_rows, all_idx
    if sample is not None and sample < len(all_idx):
        pick = np.random.default_rng(seed).choice(len(all_idx), size=sample, replace=False)
        rows, idx = all_rows[pick], all_idx[pick]
    else:
        assert len(np.unique(rows, axis=0)) == len(rows), "duplicate vector"
    h = table_hash(rows, info["hash_seed"])
    assert np.array_equal(slots[idx] & MEMO, h & MEMO), "memo differs from the row hash"
    LS = info["line_slots"]
    lines = info["capacity"] // LS
    shift = np.uint64(LS.bit_length() - 1)
    line = (h >> shift) & np.uint64(lines - 1)
    start = h & np.uint64(LS - 1)
    # line-to-line moves: double hashing (odd step from the high half),
    # linear (+1) or quadratic (the r-th move goes r lines on)
    step = (h >> np.uint64(32)) | np.uint64(1)
    probe = info["probe"]
    pending = np.ones(len(idx), dtype=bool)
    target = idx.astype(np.uint64)
    for r in range(1, lines + 1):
        if not pending.any():
            break
        for k in range(LS):
            slot = line * np.uint64(LS) + ((start + np.uint64(k)) & np.uint64(LS - 1))
            hit = pending & (slot == target)
            before = pending & ~hit
            assert np.all(slots[slot[before].astype(np.int64)] != 0), "empty slot ahead of a stored row"
            pending &= ~hit
        with np.errstate(over="ignore"):
            move = step if probe == 0 else np.uint64(1 if probe == 1 else r)
            line = (line + move) & np.uint64(lines - 1)
    assert not pending.any(), "stored row not on its probe sequence"
    return all_rows, all_idx


def check_stream_batches(o_id, n_distinct, seen, index, bounds):
    """GPU batch results vs the sequential oracle.

    For every distinct value: its first batch (in stream order) must report it
    new exactly once; every occurrence in later batches must report seen; all
    occurrences get one index; different values get different indices."""
    o_id = np.asarray(o_id)
    n = len(o_id)
    batch = np.zeros(n, dtype=np.int64)
    for b, (lo, hi) in enumerate(bounds):
        batch[lo:hi] = b
    assert bounds[-1][1] == n
    assert not np.any(seen == 0xFF), "failed operation"
    _, first_pos = np.unique(o_id, return_index=True)
    first_batch = batch[first_pos][o_id]
    later = batch > first_batch
    assert np.all(seen[later] == 1), "value from an earlier batch reported new"
    news = np.bincount(o_id[seen == 0], minlength=n_distinct)
    assert np.all(news == 1), "a value was not reported new exactly once"
    idx_of = index[first_pos]
    assert np.array_equal(index, idx_of[o_id]), "equal vectors got different indices"
    assert len(np.unique(idx_of)) == n_distinct, "different vectors share an index"
