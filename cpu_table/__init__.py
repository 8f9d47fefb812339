"""Multi-core CPU lockless table and level-synchronous BFS (cpu_table.cpp):
the paper's method on host cores, a fair multi-core CPU baseline next to the
GPU library.  Not the oracle (that one is sequential, over a library set)
and not a fallback of the GPU path (the GPU library never loads it).

* ``stream(rows, log2cap, threads)`` -> (seen u8[n], index u32[n], seconds)
* ``reach(model, cap, log2cap, threads, keep_rows=False)`` -> CpuReach
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcpu_table.so")
_lib = None


def build() -> str:
    """Compile cpu_table.cpp (host C++, -O3, pthreads) into libcpu_table.so."""
    src = os.path.join(_HERE, "cpu_table.cpp")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["g++", "-O3", "-std=c++17", "-Wall", "-pthread", "-shared", "-fPIC", src, "-o", tmp])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Summary(ctypes.Structure):
    _fields_ = [("total", ctypes.c_uint64), ("edges", ctypes.c_uint64),
                ("deadlocks", ctypes.c_uint64), ("n_levels", ctypes.c_uint32),
                ("capped", ctypes.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        L.cpu_stream.argtypes = [p, u64, u32, u32, u32, p, p, ctypes.POINTER(ctypes.c_double)]
        L.cpu_stream.restype = ctypes.c_int
        L.cpu_reach.argtypes = [p, u32, u32, u32, u32, p, u64, u32, u32, p, u32, p, u64,
                                ctypes.POINTER(_Summary), ctypes.POINTER(ctypes.c_double)]
        L.cpu_reach.restype = ctypes.c_int
        _lib = L
    return _lib


def stream(rows: np.ndarray, log2cap: int, threads: int):
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    n, W = rows.shape
    seen = np.zeros(n, dtype=np.uint8)       # touched before the timed pass
    index = np.zeros(n, dtype=np.uint32)
    sec = ctypes.c_double()
    rc = lib().cpu_stream(rows.ctypes.data, n, W, log2cap, threads, seen.ctypes.data, index.ctypes.data,
                          ctypes.byref(sec))
    if rc:
        raise RuntimeError(f"cpu_stream failed ({rc})")
    return seen, index, sec.value


@dataclasses.dataclass
class CpuReach:
    total: int
    n_levels: int
    level_counts: list
    edges: int
    deadlocks: int
    capped: bool
    seconds: float
    rows: np.ndarray | None


def reach(model, cap: int | None, log2cap: int, threads: int, keep_rows: bool = False,
          max_levels: int = 1 << 16) -> CpuReach:
    cap = model.cap if cap is None else cap
    trans = np.ascontiguousarray(model.trans, dtype=np.uint32)
    init = np.ascontiguousarray(model.init, dtype=np.uint32)
    levels = np.zeros(max_levels, dtype=np.uint64)
    max_rows = (1 << log2cap) if keep_rows else 0
    rows = np.empty((max_rows, model.W), dtype=np.uint32) if keep_rows else None
    s, sec = _Summary(), ctypes.c_double()
    rc = lib().cpu_reach(trans.ctypes.data, model.P, model.L, model.S, model.K, init.ctypes.data, cap, log2cap,
                         threads, levels.ctypes.data, max_levels, rows.ctypes.data if keep_rows else None,
                         max_rows, ctypes.byref(s), ctypes.byref(sec))
    if rc:
        raise RuntimeError(f"cpu_reach failed ({rc})")
    return CpuReach(total=s.total, n_levels=s.n_levels, level_counts=[int(x) for x in levels[:s.n_levels]],
                    edges=s.edges, deadlocks=s.deadlocks, capped=bool(s.capped), seconds=sec.value,
                    rows=rows[:s.total] if keep_rows else None)
