"""The C-ABI library loads and exports every declared symbol; host-side
argument validation fails before any device call (no GPU needed)."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from conftest import ROOT

import paper_1004_2772_amd as lhs


def _declared():
    src = open(os.path.join(ROOT, "include", "lhs.h")).read()
    return sorted(set(re.findall(r"^\s*(?:lhs_status|void|double|const char \*)\s*\**(\w+)\s*\(", src, re.M)))


def test_header_and_binding_agree():
    assert _declared() == sorted(lhs.EXPORTS)


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", lhs.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, re.M))
    missing = [s for s in _declared() if s not in exported]
    assert not missing, missing
    L = lhs.lib()
    for s in _declared():
        assert hasattr(L, s)


def test_strerror():
    L = lhs.lib()
    for code, name in lhs.STATUS.items():
        assert L.lhs_strerror(code).decode().startswith(name)


@pytest.mark.parametrize("cap,W", [(0, 4), (15, 4), (24, 4), (1 << 33, 4), (1 << 16, 0), (1 << 16, 33)])
def test_create_rejects_bad_geometry(cap, W):
    h = ctypes.c_void_p()
    assert lhs.lib().lhs_create(cap, W, ctypes.byref(h)) == 1
    assert not h.value


def test_null_handles_rejected():
    L = lhs.lib()
    n = ctypes.c_uint64()
    assert L.lhs_find_or_put(None, None, 0, None, None, None) == 1
    assert L.lhs_check(None) == 1
    assert L.lhs_count(None, ctypes.byref(n)) == 1
    assert L.lhs_dump(None, None, None, 0, ctypes.byref(n)) == 1
    assert L.lhs_clear(None, None) == 1
    assert L.lhs_destroy(None) == 0


def _bad_models():
    import gen
    good = gen.guarded_model(1, 3, 4, 2, 3, 2)
    yield "no procs", dict(P=0)
    yield "too wide", dict(P=20, S=13)
    yield "K too large", dict(K=17)
    t = good.trans.copy()
    t[0, 0, 0, 0] = 4          # target >= L
    yield "target out of range", dict(trans=t)
    t = good.trans.copy()
    t[0, 0, 0, 1] = 2          # guard var >= S
    yield "guard var out of range", dict(trans=t)
    t = good.trans.copy()
    t[0, 0, 0, 3] = 5          # effect var >= S
    yield "effect var out of range", dict(trans=t)
    t = good.trans.copy()
    t[0, 0, 0, 4] = 1 << 16    # effect value too large
    yield "effect value too large", dict(trans=t)


@pytest.mark.parametrize("name,patch", list(_bad_models()), ids=[n for n, _ in _bad_models()])
def test_reach_rejects_bad_models(name, patch):
    import gen
    g = gen.guarded_model(1, 3, 4, 2, 3, 2)
    P, L, S, K = patch.get("P", 3), 4, patch.get("S", 2), patch.get("K", 2)
    trans = np.ascontiguousarray(patch.get("trans", g.trans), dtype=np.uint32)
    init = np.zeros(max(P + S, 1), dtype=np.uint32)
    m = lhs.ReachModel(P, L, S, K, trans.ctypes.data, init.ctypes.data, 0)
    r = lhs.ReachResultC()
    assert lhs.lib().reach_explore(ctypes.byref(m), None, ctypes.byref(r)) == 1


def test_server_rejects_bad_arguments():
    L = lhs.lib()
    h = ctypes.c_void_p()
    o = lhs.ServerOpts(0, 24, 0, 0)           # capacity not a power of two
    assert L.reach_server_create(ctypes.byref(o), ctypes.byref(h)) == 1
    assert L.reach_server_create(ctypes.byref(o), None) == 1
    t = ctypes.c_uint64()
    assert L.reach_server_submit(None, None, ctypes.byref(t)) == 1
    assert L.reach_server_poll(None, 1, None, None) == 1
    assert L.reach_server_destroy(None) == 0


def test_trace_calls_reject_bad_arguments():
    import gen
    L = lhs.lib()
    n = ctypes.c_uint32()
    assert L.reach_trace(None, 0, None, None, 0, ctypes.byref(n)) == 1
    assert L.reach_deadlock_slots(None, None, 0, ctypes.byref(n)) == 1
    # predecessor records need a caller table
    m = gen.tiny_cyclic()
    st, keep = lhs._model_struct(m, None)
    o = lhs.ReachOpts(0, 0, lhs.REACH_F_PARENTS, None, None)
    r = lhs.ReachResultC()
    assert L.reach_explore(ctypes.byref(st), ctypes.byref(o), ctypes.byref(r)) == 1


def test_async_flag_conflicts_rejected():
    import gen
    L = lhs.lib()
    m = gen.tiny_cyclic()
    st, keep = lhs._model_struct(m, None)
    r = lhs.ReachResultC()
    # no levels to capture in a graph
    o = lhs.ReachOpts(0, 0, lhs.REACH_F_ASYNC | lhs.REACH_F_GRAPH, None, None)
    assert L.reach_explore(ctypes.byref(st), ctypes.byref(o), ctypes.byref(r)) == 1
    # the batch keeps levels
    arr = (ctypes.POINTER(lhs.ReachModel) * 1)(ctypes.pointer(st))
    res = (lhs.ReachResultC * 1)()
    o = lhs.ReachOpts(0, 0, lhs.REACH_F_ASYNC, None, None)
    assert L.reach_explore_batch(arr, 1, ctypes.byref(o), None, res) == 1


def test_set_workers_rejects_null():
    assert lhs.lib().lhs_set_workers(None, 4) == 1


def test_set_merge_and_counters_reject_bad_arguments():
    L = lhs.lib()
    assert L.lhs_set_merge(None, lhs.MERGE_ON) == 1
    assert L.lhs_set_counters(None, lhs.COUNT_MERGED) == 1


def test_probes_reject_bad_arguments():
    L = lhs.lib()
    fake, sink = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21)   # never dereferenced: rejected first
    assert L.lhs_probe_random_access(None, 1 << 20, 0, 1, 0, sink, None) == 1
    assert L.lhs_probe_random_access(fake, 1 << 20, 0, 1, 0, None, None) == 1
    assert L.lhs_probe_random_access(fake, 1 << 20, 3, 1, 0, sink, None) == 1          # unknown form
    assert L.lhs_probe_random_access(fake, 3 << 20, 1, 1, 0, sink, None) == 1          # rows not 2^n
    assert L.lhs_probe_random_access(ctypes.c_void_p((1 << 20) + 32), 1 << 20, 2, 1, 0, sink, None) == 1
    assert L.lhs_probe_random_lines(fake, 1 << 20, 96, 1, 1, 0, sink, None) == 1       # line width
    assert L.lhs_probe_random_cas(None, 1 << 10, 1, 0, sink, None) == 1
    assert L.lhs_probe_copy(fake, fake, 24, None) == 1                                 # not 16-byte sized


def test_binding_refuses_host_buffers_for_device_arguments():
    import torch
    host = torch.zeros(1 << 10, dtype=torch.int64)
    for call in (lambda: lhs.probe_random_access(host, "row_load", 1, 0, host),
                 lambda: lhs.probe_random_lines(np.zeros(1 << 10, np.int64), 64, 4, 1, 0, host),
                 lambda: lhs.probe_random_cas(host, 1, 0, host),
                 lambda: lhs.probe_copy(host, host)):
        with pytest.raises(ValueError):
            call()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it says so and exits non-zero
    (before touching any GPU)."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
