"""Python binding of the lhs C-ABI library (liblhs.so, HIP for gfx950).

Argument marshalling only: every step of find-or-put and of the BFS runs in
the library's kernels.  torch supplies device memory and streams; buffers are
passed as ``tensor.data_ptr()`` and streams as their ``hipStream_t`` handle.
The names follow the C header ``include/lhs.h``.

The library must be built (``python -m paper_1004_2772_amd.build``); importing
a missing library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblhs.so")
#: tuning table written by ``python -m paper_1004_2772_amd.autotune`` on the target GPU
TUNE_PATH_DEFAULT = os.path.join(PKG, "tune.json")

STATUS = {0: "LHS_OK", 1: "LHS_EINVAL", 2: "LHS_ENOMEM", 3: "LHS_EFULL", 4: "LHS_ESTALL",
          5: "LHS_EDEVICE", 6: "LHS_EBUDGET", 7: "LHS_ENOTFOUND", 8: "LHS_EAGAIN"}
REACH_NONE = 0xFFFFFFFF
REACH_F_HOST_LOOP = 1
REACH_F_GRAPH = 2
REACH_F_PARENTS = 4
REACH_F_ASYNC = 8
REACH_SERVER_F_ROUNDS = 1
COUNT_LINES = 1
COUNT_MERGED = 2
MERGE_ON = 0
MERGE_OFF = 1
MERGE_NARROW_TAGS = 2
PROBES = {"double": 0, "linear": 1, "quadratic": 2}
TUNE_TABLE, TUNE_BATCH = 0, 1

#: every symbol include/lhs.h declares
EXPORTS = ["lhs_strerror", "lhs_create", "lhs_create_ex", "lhs_get_config", "lhs_destroy",
           "lhs_clear", "lhs_find_or_put", "lhs_set_threads_per_state", "lhs_set_counters",
           "lhs_set_merge", "lhs_set_workers", "lhs_tune_load", "lhs_tune_clear", "lhs_tune_lookup",
           "lhs_check", "lhs_count", "lhs_dump", "lhs_dump_slots", "lhs_get_info",
           "reach_explore", "reach_result_free", "reach_explore_noalloc", "reach_explore_batch", "reach_trace",
           "reach_deadlock_slots",
           "reach_server_clock", "reach_server_create", "reach_server_submit", "reach_server_submit_ex",
           "reach_server_poll",
           "reach_server_wait", "reach_server_get_stats", "reach_server_destroy",
           "lhs_probe_random_lines", "lhs_probe_random_cas", "lhs_probe_random_access", "lhs_probe_copy"]


class LhsError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        self.name = STATUS.get(status, f"status {status}")
        super().__init__(f"{where}: {self.name}" if where else self.name)


class LhsInfo(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_uint64), ("state_words", ctypes.c_uint32),
                ("line_slots", ctypes.c_uint32), ("hash_seed", ctypes.c_uint64),
                ("wait_hits", ctypes.c_uint64), ("cas_failures", ctypes.c_uint64),
                ("error", ctypes.c_uint32), ("probe", ctypes.c_uint32),
                ("tps_find_or_put", ctypes.c_uint32), ("tps_expand", ctypes.c_uint32),
                ("lines_probed", ctypes.c_uint64), ("merged", ctypes.c_uint64)]


class LhsConfig(ctypes.Structure):
    _fields_ = [("line_slots", ctypes.c_uint32), ("probe", ctypes.c_uint32),
                ("tps_find_or_put", ctypes.c_uint32), ("tps_expand", ctypes.c_uint32)]


def config(line_slots: int = 16, probe="double", tps_find_or_put: int = 0,
           tps_expand: int = 0) -> LhsConfig:
    """An lhs_config; probe by name ("double", "linear", "quadratic") or number."""
    return LhsConfig(line_slots, PROBES[probe] if isinstance(probe, str) else probe,
                     tps_find_or_put, tps_expand)


def config_dict(c: LhsConfig) -> dict:
    names = {v: k for k, v in PROBES.items()}
    return {"line_slots": c.line_slots, "probe": names.get(c.probe, c.probe),
            "tps_find_or_put": c.tps_find_or_put, "tps_expand": c.tps_expand}


class ReachModel(ctypes.Structure):
    _fields_ = [("n_procs", ctypes.c_uint32), ("n_locals", ctypes.c_uint32),
                ("n_shared", ctypes.c_uint32), ("trans_per_local", ctypes.c_uint32),
                ("trans", ctypes.c_void_p), ("init", ctypes.c_void_p),
                ("state_cap", ctypes.c_uint64)]


class ReachOpts(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_uint64), ("max_levels", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("table", ctypes.c_void_p),
                ("hip_stream", ctypes.c_void_p)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("capacity", ctypes.c_uint64),
                ("max_active", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("table", LhsConfig)]


class QueryTimes(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("done_s", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("steps", ctypes.c_uint64), ("states", ctypes.c_uint64),
                ("bytes_in_use", ctypes.c_uint64), ("bytes_pooled", ctypes.c_uint64),
                ("peak_bytes", ctypes.c_uint64), ("active", ctypes.c_uint32),
                ("queued", ctypes.c_uint32), ("busy_s", ctypes.c_double)]


class ReachResultC(ctypes.Structure):
    _fields_ = [("total_states", ctypes.c_uint64), ("edges", ctypes.c_uint64),
                ("deadlocks", ctypes.c_uint64), ("wait_hits", ctypes.c_uint64),
                ("level_counts", ctypes.POINTER(ctypes.c_uint64)), ("n_levels", ctypes.c_uint32),
                ("capped", ctypes.c_int32), ("gpu_ms", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load liblhs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1004_2772_amd.build`")
        # torch's HIP runtime first: started by the library instead, it
        # leaves torch without a GPU in this process
        try:
            import torch
            torch.cuda.is_available()
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        u64, u32, p, st = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
        L.lhs_strerror.argtypes = [st]
        L.lhs_strerror.restype = ctypes.c_char_p
        L.lhs_create.argtypes = [u64, u32, ctypes.POINTER(p)]
        L.lhs_create_ex.argtypes = [u64, u32, ctypes.POINTER(LhsConfig), ctypes.POINTER(p)]
        L.lhs_get_config.argtypes = [p, ctypes.POINTER(LhsConfig)]
        L.lhs_tune_load.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(u32)]
        L.lhs_tune_clear.argtypes = []
        L.lhs_tune_lookup.argtypes = [u32, u32, u64, ctypes.POINTER(LhsConfig),
                                      ctypes.POINTER(ctypes.c_int32)]
        L.lhs_destroy.argtypes = [p]
        L.lhs_clear.argtypes = [p, p]
        L.lhs_find_or_put.argtypes = [p, p, u64, p, p, p]
        L.lhs_check.argtypes = [p]
        L.lhs_set_threads_per_state.argtypes = [p, u32]
        L.lhs_set_counters.argtypes = [p, u32]
        L.lhs_set_workers.argtypes = [p, u32]
        L.lhs_set_merge.argtypes = [p, u32]
        L.lhs_count.argtypes = [p, ctypes.POINTER(u64)]
        L.lhs_dump.argtypes = [p, p, p, u64, ctypes.POINTER(u64)]
        L.lhs_dump_slots.argtypes = [p, p]
        L.lhs_get_info.argtypes = [p, ctypes.POINTER(LhsInfo)]
        L.reach_explore.argtypes = [ctypes.POINTER(ReachModel), ctypes.POINTER(ReachOpts),
                                    ctypes.POINTER(ReachResultC)]
        L.reach_result_free.argtypes = [ctypes.POINTER(ReachResultC)]
        L.reach_explore_noalloc.argtypes = [ctypes.POINTER(ReachModel), p, p, u32,
                                            ctypes.POINTER(ReachResultC), p]
        L.reach_trace.argtypes = [p, u32, p, p, u32, ctypes.POINTER(u32)]
        L.reach_deadlock_slots.argtypes = [p, p, u32, ctypes.POINTER(u32)]
        L.reach_explore_batch.argtypes = [ctypes.POINTER(ctypes.POINTER(ReachModel)), u32,
                                          ctypes.POINTER(ReachOpts), ctypes.POINTER(p),
                                          ctypes.POINTER(ReachResultC)]
        L.reach_result_free.restype = None
        L.reach_server_clock.argtypes = []
        L.reach_server_clock.restype = ctypes.c_double
        L.reach_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(p)]
        L.reach_server_submit.argtypes = [p, ctypes.POINTER(ReachModel), ctypes.POINTER(u64)]
        L.reach_server_submit_ex.argtypes = [p, ctypes.POINTER(ReachModel), p, ctypes.POINTER(u64)]
        L.reach_server_poll.argtypes = [p, u64, ctypes.POINTER(ReachResultC), ctypes.POINTER(QueryTimes)]
        L.reach_server_wait.argtypes = [p, u64, ctypes.POINTER(ReachResultC), ctypes.POINTER(QueryTimes)]
        L.reach_server_get_stats.argtypes = [p, ctypes.POINTER(ServerStats)]
        L.reach_server_destroy.argtypes = [p]
        L.lhs_probe_random_lines.argtypes = [p, u64, u32, u32, u64, u64, p, p]
        L.lhs_probe_random_cas.argtypes = [p, u64, u64, u64, p, p]
        L.lhs_probe_random_access.argtypes = [p, u64, u32, u64, u64, p, p]
        L.lhs_probe_copy.argtypes = [p, p, u64, p]
        for name in ("lhs_probe_random_lines", "lhs_probe_random_cas", "lhs_probe_random_access", "lhs_probe_copy",
                     "lhs_create", "lhs_destroy", "lhs_clear", "lhs_find_or_put", "lhs_check",
                     "lhs_set_threads_per_state", "lhs_set_counters", "lhs_set_merge", "lhs_set_workers",
                     "lhs_create_ex",
                     "lhs_get_config",
                     "lhs_tune_load", "lhs_tune_clear", "lhs_tune_lookup",
                     "lhs_count", "lhs_dump", "lhs_dump_slots", "lhs_get_info", "reach_explore",
                     "reach_explore_noalloc",
                     "reach_explore_batch", "reach_trace", "reach_deadlock_slots",
                     "reach_server_create", "reach_server_submit", "reach_server_submit_ex",
                     "reach_server_poll", "reach_server_wait", "reach_server_get_stats",
                     "reach_server_destroy"):
            getattr(L, name).restype = st
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != 0:
        raise LhsError(rc, where)


def _stream_handle(stream) -> int | None:
    """hipStream_t of a torch stream (None -> torch's current stream)."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _ptr(x) -> int | None:
    """Device/host address of a torch tensor or numpy array (None passes through)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data
    if not x.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return x.data_ptr()


def _dptr(x, what: str) -> int | None:
    """Address of a contiguous GPU tensor (None passes through); anything else
    is refused before it reaches a kernel as a device address."""
    if x is None:
        return None
    if isinstance(x, np.ndarray) or not getattr(x, "is_cuda", False):
        raise ValueError(f"{what} must be a GPU tensor")
    if not x.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return x.data_ptr()


def tune_load(path: str, device: str | None = None) -> int:
    """Load a tuning file (lhs_tune_load); returns the entries kept."""
    n = ctypes.c_uint32()
    _check(lib().lhs_tune_load(os.fsencode(path), device.encode() if device else None,
                               ctypes.byref(n)), "lhs_tune_load")
    return n.value


def tune_load_default() -> int:
    """Load the tuning table named by the LHS_TUNE_FILE environment variable,
    else the package's own if it exists; returns the entries kept (0 if there
    is none or it was measured on another device)."""
    path = os.environ.get("LHS_TUNE_FILE") or TUNE_PATH_DEFAULT
    if not os.path.exists(path):
        return 0
    return tune_load(path)


def tune_clear():
    _check(lib().lhs_tune_clear(), "lhs_tune_clear")


def tune_lookup(kind: int, state_words: int, capacity: int):
    """(config dict, found) the tuning table gives for a table (lhs_tune_lookup)."""
    c, f = LhsConfig(), ctypes.c_int32()
    _check(lib().lhs_tune_lookup(kind, state_words, capacity, ctypes.byref(c), ctypes.byref(f)),
           "lhs_tune_lookup")
    return config_dict(c), bool(f.value)


class Table:
    """A lockless find-or-put table on the current HIP device.  ``cfg``: an
    LhsConfig (lhs_create_ex) or None for lhs_create (tuned or default)."""

    def __init__(self, capacity: int, state_words: int, cfg: LhsConfig | None = None):
        h = ctypes.c_void_p()
        if cfg is None:
            _check(lib().lhs_create(capacity, state_words, ctypes.byref(h)), "lhs_create")
        else:
            _check(lib().lhs_create_ex(capacity, state_words, ctypes.byref(cfg), ctypes.byref(h)),
                   "lhs_create_ex")
        self.handle = h
        self.capacity = capacity
        self.W = state_words

    def close(self):
        if self.handle:
            lib().lhs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def clear(self, stream=None):
        _check(lib().lhs_clear(self.handle, _stream_handle(stream)), "lhs_clear")

    def find_or_put(self, states, seen, index=None, stream=None):
        """states: device tensor [n, W] (32-bit); seen: device uint8 [n];
        index: device 32-bit [n] or None.  Asynchronous on ``stream``."""
        n = states.shape[0] if states.dim() == 2 else 0
        if states.dim() != 2 or states.shape[1] != self.W or states.element_size() != 4:
            raise ValueError("states must be a [n, W] tensor of 32-bit words")
        if seen.numel() < n or seen.element_size() != 1:
            raise ValueError("seen must hold n bytes")
        if index is not None and (index.numel() < n or index.element_size() != 4):
            raise ValueError("index must hold n 32-bit words")
        _check(lib().lhs_find_or_put(self.handle, _dptr(states, "states"), n, _dptr(seen, "seen"),
                                     _dptr(index, "index"),
                                     _stream_handle(stream)), "lhs_find_or_put")

    def check(self):
        _check(lib().lhs_check(self.handle), "lhs_check")

    def set_threads_per_state(self, tps: int):
        _check(lib().lhs_set_threads_per_state(self.handle, tps), "lhs_set_threads_per_state")

    def set_counters(self, flags: int):
        """LHS_COUNT_LINES (1): count lines probed (lhs_info.lines_probed);
        LHS_COUNT_MERGED (2): count successors merged in expansion passes
        (lhs_info.merged)."""
        _check(lib().lhs_set_counters(self.handle, flags), "lhs_set_counters")

    def set_merge(self, mode: int):
        """MERGE_ON (default), MERGE_OFF or MERGE_NARROW_TAGS: how explorations
        on this table treat equal successors of one expansion pass."""
        _check(lib().lhs_set_merge(self.handle, mode), "lhs_set_merge")

    def set_workers(self, max_workgroups: int):
        """At most this many workgroups expand states in explorations on this
        table (0 = all that fit on the GPU at once)."""
        _check(lib().lhs_set_workers(self.handle, max_workgroups), "lhs_set_workers")

    def count(self) -> int:
        c = ctypes.c_uint64()
        _check(lib().lhs_count(self.handle, ctypes.byref(c)), "lhs_count")
        return c.value

    def dump(self):
        """(rows u32 [n, W], slots u32 [n]) of every stored vector, by slot."""
        n = ctypes.c_uint64()
        _check(lib().lhs_dump(self.handle, None, None, 0, ctypes.byref(n)), "lhs_dump")
        rows = np.empty((n.value, self.W), dtype=np.uint32)
        idx = np.empty(n.value, dtype=np.uint32)
        if n.value:
            _check(lib().lhs_dump(self.handle, _ptr(rows), _ptr(idx), n.value, ctypes.byref(n)),
                   "lhs_dump")
        return rows, idx

    def dump_slots(self) -> np.ndarray:
        out = np.empty(self.capacity, dtype=np.uint64)
        _check(lib().lhs_dump_slots(self.handle, _ptr(out)), "lhs_dump_slots")
        return out

    def info(self) -> dict:
        i = LhsInfo()
        _check(lib().lhs_get_info(self.handle, ctypes.byref(i)), "lhs_get_info")
        return {f: getattr(i, f) for f, _ in LhsInfo._fields_}

    def trace(self, slot: int):
        """(slots [n], rows [n, W]) from s0 to the state in `slot` (needs the
        last reach_explore on this table to have used REACH_F_PARENTS)."""
        n = ctypes.c_uint32()
        _check(lib().reach_trace(self.handle, slot, None, None, 0, ctypes.byref(n)), "reach_trace")
        path = np.empty(n.value, dtype=np.uint32)
        rows = np.empty((n.value, self.W), dtype=np.uint32)
        _check(lib().reach_trace(self.handle, slot, _ptr(path), _ptr(rows), n.value, ctypes.byref(n)),
               "reach_trace")
        return path, rows

    def deadlock_slots(self):
        """(number of deadlock states expanded, slots of the first <= 1024)."""
        n = ctypes.c_uint32()
        _check(lib().reach_deadlock_slots(self.handle, None, 0, ctypes.byref(n)), "reach_deadlock_slots")
        out = np.empty(min(n.value, 1024), dtype=np.uint32)
        _check(lib().reach_deadlock_slots(self.handle, _ptr(out), len(out), ctypes.byref(n)),
               "reach_deadlock_slots")
        return n.value, out

    def config(self) -> dict:
        c = LhsConfig()
        _check(lib().lhs_get_config(self.handle, ctypes.byref(c)), "lhs_get_config")
        return config_dict(c)


@dataclasses.dataclass
class ReachResult:
    total: int
    n_levels: int
    level_counts: list
    edges: int
    deadlocks: int
    capped: bool
    wait_hits: int
    gpu_ms: float


def _model_struct(model, cap):
    """ReachModel over model.trans [P, L, K, 5] and model.init (kept alive by caller)."""
    trans = np.ascontiguousarray(model.trans, dtype=np.uint32)
    if trans.shape != (model.P, model.L, model.K, 5):
        raise ValueError("trans must be [P, L, K, 5]")
    init = np.ascontiguousarray(model.init, dtype=np.uint32)
    if init.shape != (model.P + model.S,):
        raise ValueError("init must have P + S words")
    m = ReachModel(model.P, model.L, model.S, model.K, trans.ctypes.data, init.ctypes.data,
                   model.cap if cap is None else cap)
    return m, (trans, init)


def _result(r: ReachResultC) -> ReachResult:
    levels = [int(r.level_counts[i]) for i in range(r.n_levels)]
    return ReachResult(total=r.total_states, n_levels=r.n_levels, level_counts=levels,
                       edges=r.edges, deadlocks=r.deadlocks, capped=bool(r.capped),
                       wait_hits=r.wait_hits, gpu_ms=r.gpu_ms)


def reach_explore_batch(models, capacity: int = 0, tables=None, stream=None, max_levels: int = 0,
                        flags: int = 0, caps=None) -> list:
    """Explore several models together on the GPU (synchronous).  ``tables``:
    optional list of Table (or None) per model; ``caps``: optional per-model
    state caps overriding model.cap."""
    n = len(models)
    structs, keep = [], []
    for i, m in enumerate(models):
        st, k = _model_struct(m, None if caps is None else caps[i])
        structs.append(st)
        keep.append(k)
    arr = (ctypes.POINTER(ReachModel) * n)(*[ctypes.pointer(x) for x in structs])
    tabs = None
    if tables is not None:
        tabs = (ctypes.c_void_p * n)(*[(t.handle.value if t is not None else None) for t in tables])
    o = ReachOpts(capacity, max_levels, flags, None, _stream_handle(stream))
    res = (ReachResultC * n)()
    _check(lib().reach_explore_batch(arr, n, ctypes.byref(o),
                                     ctypes.cast(tabs, ctypes.POINTER(ctypes.c_void_p)) if tabs else None,
                                     res), "reach_explore_batch")
    try:
        return [_result(res[i]) for i in range(n)]
    finally:
        for i in range(n):
            lib().reach_result_free(ctypes.byref(res[i]))
        del keep, structs


def reach_explore(model, cap: int | None = None, capacity: int = 0, table: Table | None = None,
                  stream=None, max_levels: int = 0, flags: int = 0) -> ReachResult:
    """Level-synchronous BFS of ``model`` on the GPU (synchronous); with
    flags=REACH_F_ASYNC the exploration without level barriers (no level
    counts: n_levels 0).

    model: object with P, L, S, K, trans [P, L, K, 5] (uint32, 0xFFFFFFFF = none),
    init [P + S]; cap overrides model.cap (0 = none)."""
    m, keep = _model_struct(model, cap)
    o = ReachOpts(capacity, max_levels, flags, table.handle if table else None,
                  _stream_handle(stream))
    r = ReachResultC()
    _check(lib().reach_explore(ctypes.byref(m), ctypes.byref(o), ctypes.byref(r)), "reach_explore")
    try:
        levels = [int(r.level_counts[i]) for i in range(r.n_levels)]
        return ReachResult(total=r.total_states, n_levels=r.n_levels, level_counts=levels,
                           edges=r.edges, deadlocks=r.deadlocks, capped=bool(r.capped),
                           wait_hits=r.wait_hits, gpu_ms=r.gpu_ms)
    finally:
        lib().reach_result_free(ctypes.byref(r))
        del keep


#: limits of reach_explore_noalloc (include/lhs.h)
NOALLOC_MAX_CAPACITY = 1 << 21
NOALLOC_MAX_TRANS = 1 << 16


def reach_explore_noalloc(model, table: Table, cap: int | None = None, max_levels: int = 1 << 16,
                          stream=None) -> ReachResult:
    """reach_explore on ``table`` through the entry point that allocates
    nothing (reach_explore_noalloc); the level counts land in a host array
    this binding passes in."""
    m, keep = _model_struct(model, cap)
    levels = np.zeros(max_levels, dtype=np.uint64)
    r = ReachResultC()
    _check(lib().reach_explore_noalloc(ctypes.byref(m), table.handle, _ptr(levels), max_levels,
                                       ctypes.byref(r), _stream_handle(stream)), "reach_explore_noalloc")
    del keep
    return ReachResult(total=r.total_states, n_levels=r.n_levels,
                       level_counts=[int(x) for x in levels[: r.n_levels]], edges=r.edges,
                       deadlocks=r.deadlocks, capped=bool(r.capped), wait_hits=r.wait_hits, gpu_ms=r.gpu_ms)


class Server:
    """Continuous-batching reachability server (one worker thread on the GPU):
    one persistent launch serves every query, or with ``rounds`` the host
    launches rounds of level steps (REACH_SERVER_F_ROUNDS)."""

    def __init__(self, budget_bytes: int = 0, capacity: int = 0, max_active: int = 0,
                 cfg: LhsConfig | None = None, rounds: bool = False):
        h = ctypes.c_void_p()
        o = ServerOpts(budget_bytes, capacity, max_active, REACH_SERVER_F_ROUNDS if rounds else 0,
                       cfg if cfg is not None else LhsConfig())
        _check(lib().reach_server_create(ctypes.byref(o), ctypes.byref(h)), "reach_server_create")
        self.handle = h

    @staticmethod
    def clock() -> float:
        return lib().reach_server_clock()

    def submit(self, model, cap: int | None = None, table: Table | None = None) -> int:
        """Queue a query; with ``table`` it runs on that table, which keeps
        the query's reachable set once collected (reach_server_submit_ex)."""
        m, keep = _model_struct(model, cap)
        t = ctypes.c_uint64()
        if table is None:
            _check(lib().reach_server_submit(self.handle, ctypes.byref(m), ctypes.byref(t)),
                   "reach_server_submit")
        else:
            _check(lib().reach_server_submit_ex(self.handle, ctypes.byref(m), table.handle, ctypes.byref(t)),
                   "reach_server_submit_ex")
        del keep
        return t.value

    def _collect(self, fn, ticket):
        r, tm = ReachResultC(), QueryTimes()
        rc = fn(self.handle, ticket, ctypes.byref(r), ctypes.byref(tm))
        if rc == 8:          # LHS_EAGAIN
            return None
        try:
            _check(rc, "reach_server_poll")
            return _result(r), (tm.submit_s, tm.admit_s, tm.done_s)
        finally:
            lib().reach_result_free(ctypes.byref(r))

    def poll(self, ticket: int):
        """(ReachResult, (submit_s, admit_s, done_s)) or None while running."""
        return self._collect(lib().reach_server_poll, ticket)

    def wait(self, ticket: int):
        return self._collect(lib().reach_server_wait, ticket)

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().reach_server_get_stats(self.handle, ctypes.byref(st)), "reach_server_get_stats")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self.handle:
            rc = lib().reach_server_destroy(self.handle)
            self.handle = None
            _check(rc, "reach_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def probe_random_lines(buf, line_bytes: int, lanes_per_line: int, n_reads: int, seed: int, sink,
                       stream=None):
    _check(lib().lhs_probe_random_lines(_dptr(buf, "buf"), buf.numel() * buf.element_size(), line_bytes,
                                        lanes_per_line, n_reads, seed, _dptr(sink, "sink"),
                                        _stream_handle(stream)), "lhs_probe_random_lines")


def probe_random_cas(slots, n_ops: int, seed: int, sink, stream=None):
    _check(lib().lhs_probe_random_cas(_dptr(slots, "slots"), slots.numel(), n_ops, seed, _dptr(sink, "sink"),
                                      _stream_handle(stream)), "lhs_probe_random_cas")


PROBE_FORMS = {"slot_store": 0, "row_store": 1, "row_load": 2}


def probe_random_access(buf, form, n_ops: int, seed: int, sink, stream=None):
    """form: "slot_store", "row_store", "row_load" (or its number)."""
    f = PROBE_FORMS[form] if isinstance(form, str) else form
    _check(lib().lhs_probe_random_access(_dptr(buf, "buf"), buf.numel() * buf.element_size(), f, n_ops, seed,
                                         _dptr(sink, "sink"), _stream_handle(stream)), "lhs_probe_random_access")


def probe_copy(dst, src, stream=None):
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    _check(lib().lhs_probe_copy(_dptr(dst, "dst"), _dptr(src, "src"), nbytes, _stream_handle(stream)), "lhs_probe_copy")
