"""Tuning table (lhs_tune_load / lhs_tune_lookup) and table-shape validation:
host-only calls of the C-ABI, no GPU needed."""
import ctypes
import json

import pytest

import paper_1004_2772_amd as lhs

DEFAULT = {"line_slots": 16, "probe": "double", "tps_find_or_put": 0, "tps_expand": 0}


def _entry(kind, W, lc, ls, probe, tf, te, **extra):
    e = {"kind": kind, "W": W, "log2_capacity": lc, "line_slots": ls, "probe": probe,
         "tps_find_or_put": tf, "tps_expand": te}
    e.update(extra)
    return e


ENTRIES = [
    _entry("table", 4, 20, 8, "linear", 1, 4, stream_ms={"a": 1.5}),
    _entry("table", 4, 28, 16, "double", 4, 1),
    _entry("table", 16, 20, 32, "quadratic", 8, 8),
    _entry("table", 16, 24, 16, "linear", 16, 1),
    _entry("table", 16, 28, 8, "double", 4, 16),
    _entry("batch", 32, 21, 32, "linear", 0, 4),
]


def _write(tmp_path, obj, name="tune.json"):
    p = tmp_path / name
    p.write_text(obj if isinstance(obj, str) else json.dumps(obj))
    return str(p)


@pytest.fixture
def loaded(tmp_path):
    doc = {"format": "lhs-tune-1", "device": "gfx950", "note": "café \\\"q\\\" ☃",
           "entries": ENTRIES}
    n = lhs.tune_load(_write(tmp_path, doc), device="gfx950")
    assert n == len(ENTRIES)
    yield
    lhs.tune_clear()


def _cfg(e):
    return {k: e[k] for k in ("line_slots", "probe", "tps_find_or_put", "tps_expand")}


@pytest.mark.parametrize("W,cap,want", [
    (4, 1 << 20, 0),      # exact
    (3, 1 << 21, 0),      # smallest tuned W >= 3 is 4; 21 is nearest to 20
    (4, 1 << 24, 1),      # 24 is as near to 20 as to 28: the larger wins
    (4, 1 << 32, 1),
    (5, 1 << 16, 2),      # W 5..16 -> the W=16 entries
    (16, 1 << 23, 3),
    (16, 1 << 26, 4),     # as near to 24 as to 28: the larger wins
    (9, 1 << 27, 4),
    (32, 1 << 20, 2),     # wider than every entry: the largest tuned W (16)
])
def test_lookup_rules(loaded, W, cap, want):
    cfg, found = lhs.tune_lookup(lhs.TUNE_TABLE, W, cap)
    assert found
    assert cfg == _cfg(ENTRIES[want])


def test_kinds_are_separate(loaded):
    cfg, found = lhs.tune_lookup(lhs.TUNE_BATCH, 7, 1 << 21)
    assert found and cfg == _cfg(ENTRIES[5])


def test_no_table_gives_defaults():
    lhs.tune_clear()
    cfg, found = lhs.tune_lookup(lhs.TUNE_TABLE, 16, 1 << 28)
    assert not found and cfg == DEFAULT


def test_other_device_entries_are_skipped(tmp_path):
    doc = {"format": "lhs-tune-1", "device": "gfx942", "entries": ENTRIES}
    assert lhs.tune_load(_write(tmp_path, doc), device="gfx950") == 0
    cfg, found = lhs.tune_lookup(lhs.TUNE_TABLE, 16, 1 << 28)
    assert not found and cfg == DEFAULT


BAD = [
    "{",                                                         # truncated
    '{"format": "lhs-tune-1", "device": "gfx950", "entries": []} x',   # trailing garbage
    '{"format": "lhs-tune-2", "device": "gfx950", "entries": []}',     # unknown format
    '{"format": "lhs-tune-1", "device": "gfx950"}',                    # no entries
    '{"format": "lhs-tune-1", "device": "gfx950", "entries": [1]}',    # entry not an object
    '{"format": "lhs-tune-1", "device": "gfx950", "entries": [], }',   # trailing comma
    '["format"]',
    '{"format": "lhs-tune-1", "device": "gfx950", "entries": [{"kind": "table"}]}',
]


def _bad_entries():
    for field, value in [("line_slots", 12), ("line_slots", 64), ("tps_find_or_put", 2),
                         ("tps_expand", 32), ("probe", "cubic"), ("kind", "other"), ("W", 0),
                         ("W", 33), ("log2_capacity", 40), ("W", 4.5), ("W", -4), ("W", "4")]:
        e = dict(ENTRIES[0])
        e[field] = value
        yield f"{field}={value!r}", json.dumps({"format": "lhs-tune-1", "device": "gfx950", "entries": [e]})


@pytest.mark.parametrize("text", BAD + [t for _, t in _bad_entries()],
                         ids=[f"bad{i}" for i in range(len(BAD))] + [n for n, _ in _bad_entries()])
def test_malformed_files_rejected_and_table_kept(loaded, tmp_path, text):
    with pytest.raises(lhs.LhsError) as ei:
        lhs.tune_load(_write(tmp_path, text, "bad.json"), device="gfx950")
    assert ei.value.name == "LHS_EINVAL"
    cfg, found = lhs.tune_lookup(lhs.TUNE_TABLE, 4, 1 << 20)     # previous table still loaded
    assert found and cfg == _cfg(ENTRIES[0])


def test_missing_file_rejected(tmp_path):
    with pytest.raises(lhs.LhsError):
        lhs.tune_load(str(tmp_path / "nope.json"), device="gfx950")


def test_lookup_rejects_bad_arguments():
    L = lhs.lib()
    c = lhs.LhsConfig()
    assert L.lhs_tune_lookup(2, 4, 1024, ctypes.byref(c), None) == 1
    assert L.lhs_tune_lookup(0, 0, 1024, ctypes.byref(c), None) == 1
    assert L.lhs_tune_lookup(0, 33, 1024, ctypes.byref(c), None) == 1
    assert L.lhs_tune_lookup(0, 4, 1024, None, None) == 1
    assert L.lhs_tune_load(None, None, None) == 1


@pytest.mark.parametrize("cfg", [
    lhs.LhsConfig(12, 0, 0, 0), lhs.LhsConfig(64, 0, 0, 0), lhs.LhsConfig(16, 3, 0, 0),
    lhs.LhsConfig(16, 0, 2, 0), lhs.LhsConfig(16, 0, 0, 32),
])
def test_create_ex_rejects_bad_shapes(cfg):
    h = ctypes.c_void_p()
    assert lhs.lib().lhs_create_ex(1 << 16, 4, ctypes.byref(cfg), ctypes.byref(h)) == 1
    assert not h.value


def test_create_ex_rejects_capacity_below_line():
    h = ctypes.c_void_p()
    cfg = lhs.LhsConfig(32, 0, 0, 0)
    assert lhs.lib().lhs_create_ex(16, 4, ctypes.byref(cfg), ctypes.byref(h)) == 1


def test_server_rejects_bad_shape():
    h = ctypes.c_void_p()
    o = lhs.ServerOpts(0, 0, 0, 0, lhs.LhsConfig(24, 0, 0, 0))
    assert lhs.lib().reach_server_create(ctypes.byref(o), ctypes.byref(h)) == 1
    assert not h.value


def _times(best, others=1.10, tweak=None):
    from paper_1004_2772_amd import autotune
    t = {autotune._key(ls, p, g): others for ls in autotune.LINES for p in autotune.PROBE_NAMES
         for g in autotune.TPS}
    for k, v in (tweak or {}).items():
        t[k] = v
    t[best] = 1.0
    return t


def test_autotune_prefers_double_hashing_within_tolerance():
    from paper_1004_2772_amd import autotune
    # linear is best by 1 %: double hashing at the same line width wins
    a = _times("8/linear/1", tweak={"8/double/4": 1.01})
    b = _times("8/linear/4", tweak={"8/double/1": 1.005})
    (ls, probe, ta, tb), _ = autotune.choose(a, b)
    assert (ls, probe, ta, tb) == (8, "double", 4, 1)
    # by more than the tolerance the faster probe sequence is kept
    a = _times("16/linear/1", tweak={"16/double/1": 1.2})
    (ls, probe, ta, tb), _ = autotune.choose(a, None)
    assert (ls, probe, ta) == (16, "linear", 1)


def test_autotune_reselect_keeps_format(tmp_path):
    import shutil

    from paper_1004_2772_amd import TUNE_PATH_DEFAULT, autotune
    p = tmp_path / "tune.json"
    shutil.copy(TUNE_PATH_DEFAULT, p)
    doc = autotune.reselect(str(p))
    assert lhs.tune_load(str(p), device=doc["device"]) == len(doc["entries"])
    lhs.tune_clear()
