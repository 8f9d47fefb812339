"""CPU oracle for the reachability hot path — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  The GPU library never loads it and shares no
code with it; both read the arrays produced by ``gen``.

Contents
--------
* ``reach``      — sequential level-synchronous BFS over a std::unordered_set
                   (oracle.cpp; Algorithm 1 with the queue-if-new reading).
* ``stream``     — sequential find-or-put over a stream (Algorithm 3's
                   contract: seen = row occurred before; id = first-occurrence
                   ordinal).
* ``successors`` — next-state of one state, for sampled checks at full size.
* ``digest``     — order-independent set digest (count, sum, xor).
* ``brute``      — brute-force product enumeration with distance relaxation
                   (an independent algorithm used to pin ``reach``).
* ``closed_form``— exact level counts of N independent cyclic L-state
                   processes (another pin).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile oracle.cpp (host C++, -O2) into liboracle.so."""
    src = os.path.join(_HERE, "oracle.cpp")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-Wall", "-shared", "-fPIC", src, "-o", tmp])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Summary(ctypes.Structure):
    _fields_ = [("total", ctypes.c_uint64), ("edges", ctypes.c_uint64),
                ("deadlocks", ctypes.c_uint64), ("digest_sum", ctypes.c_uint64),
                ("digest_xor", ctypes.c_uint64), ("n_levels", ctypes.c_uint32),
                ("capped", ctypes.c_int32)]


def load(path: str):
    """Load a compiled oracle library and declare its C signatures."""
    L = ctypes.CDLL(path)
    u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
    L.oracle_reach.argtypes = [p, u32, u32, u32, u32, p, u64, p, u32, p, u64,
                               ctypes.POINTER(_Summary)]
    L.oracle_reach.restype = ctypes.c_int
    L.oracle_successors.argtypes = [p, u32, u32, u32, u32, p, p, u64]
    L.oracle_successors.restype = ctypes.c_int64
    L.oracle_stream.argtypes = [p, u64, u32, p, p]
    L.oracle_stream.restype = u64
    L.oracle_digest.argtypes = [p, u64, u32, ctypes.POINTER(u64), ctypes.POINTER(u64)]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = load(_LIB_PATH)
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


@dataclasses.dataclass
class ReachResult:
    total: int
    n_levels: int
    level_counts: list
    edges: int
    deadlocks: int
    capped: bool
    digest: tuple          # (count, sum, xor)
    states: np.ndarray | None = None   # [total, W] in BFS order, if requested


def reach(model, cap: int | None = None, keep_states: bool = False,
          max_levels: int = 1 << 20) -> ReachResult:
    """Sequential BFS of ``model`` (a gen.Model).  ``cap`` overrides model.cap."""
    cap = model.cap if cap is None else cap
    trans = np.ascontiguousarray(model.trans, dtype=np.uint32)
    init = np.ascontiguousarray(model.init, dtype=np.uint32)
    levels = np.zeros(max_levels, dtype=np.uint64)
    s = _Summary()
    out = None
    out_rows = 0
    if keep_states:
        # upper bound for the buffer: cap if given, else run twice
        if cap:
            out_rows = cap
            out = np.empty((out_rows, model.W), dtype=np.uint32)
    rc = lib().oracle_reach(_ptr(trans), model.P, model.L, model.S, model.K, _ptr(init),
                            cap, _ptr(levels), max_levels,
                            _ptr(out) if out is not None else None, out_rows, ctypes.byref(s))
    if rc != 0:
        raise RuntimeError(f"oracle_reach failed rc={rc}")
    if keep_states and out is None:
        out = np.empty((s.total, model.W), dtype=np.uint32)
        rc = lib().oracle_reach(_ptr(trans), model.P, model.L, model.S, model.K, _ptr(init),
                                cap, _ptr(levels), max_levels, _ptr(out), s.total,
                                ctypes.byref(s))
        assert rc == 0
    states = out[: s.total] if keep_states else None
    return ReachResult(total=s.total, n_levels=s.n_levels,
                       level_counts=[int(x) for x in levels[: s.n_levels]],
                       edges=s.edges, deadlocks=s.deadlocks, capped=bool(s.capped),
                       digest=(s.total, s.digest_sum, s.digest_xor), states=states)


def successors(model, state) -> np.ndarray:
    trans = np.ascontiguousarray(model.trans, dtype=np.uint32)
    st = np.ascontiguousarray(state, dtype=np.uint32)
    cap = model.P * model.K
    out = np.empty((max(cap, 1), model.W), dtype=np.uint32)
    n = lib().oracle_successors(_ptr(trans), model.P, model.L, model.S, model.K, _ptr(st),
                                _ptr(out), cap)
    if n < 0:
        raise RuntimeError("successor buffer too small")
    return out[:n]


def stream(rows: np.ndarray):
    """Sequential find-or-put over rows [n, W]: (seen u8[n], id u32[n], n_distinct)."""
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    n, W = rows.shape
    seen = np.empty(n, dtype=np.uint8)
    ids = np.empty(n, dtype=np.uint32)
    d = lib().oracle_stream(_ptr(rows), n, W, _ptr(seen), _ptr(ids))
    return seen, ids, int(d)


def digest(rows: np.ndarray) -> tuple:
    """(count, sum, xor) of the oracle's row digest over rows [n, W]."""
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    n, W = rows.shape if rows.ndim == 2 else (0, 1)
    s, x = ctypes.c_uint64(), ctypes.c_uint64()
    if n:
        lib().oracle_digest(_ptr(rows), n, W, ctypes.byref(s), ctypes.byref(x))
    return (n, s.value, x.value)
