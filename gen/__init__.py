"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

Nothing here computes reachability, hashing or probing: the module only draws
random numbers (xorshift64, Marsaglia 2003) and lays them out as transition
tables of synthetic models and as shuffled duplicate streams.  The native part
is ``gen/gen.c`` (built into ``gen/libgen.so``); this file marshals arrays.

Models follow the explicit-state setting of the paper (Preliminaries section:
a model yields an initial state and a next-state function).  A model has P
interleaved processes with L local states each, S shared variables with values
below D, and K guarded transitions per (process, local state).  The state
vector has W = P + S words: the P local states, then the S shared values.
"""
from __future__ import annotations

import ctypes
import dataclasses
import json
import os
import subprocess

import numpy as np

NONE = 0xFFFFFFFF
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgen.so")
_lib = None


def build() -> str:
    """Compile gen.c into libgen.so (host C, gcc)."""
    src = os.path.join(_HERE, "gen.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-Wall", "-shared", "-fPIC", src, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        L.gen_xs64.argtypes = [u64, p, u64]
        L.gen_words.argtypes = [u64, p, u64]
        L.gen_guarded_model.argtypes = [u64, u32, u32, u32, u32, u32, p]
        L.gen_guarded_model.restype = ctypes.c_int
        L.gen_cyclic_model.argtypes = [u32, u32, p]
        L.gen_cyclic_model.restype = ctypes.c_int
        L.gen_permutation.argtypes = [u64, p, u64]
        L.gen_dup_stream.argtypes = [u64, u64, u32, u32, p, p]
        L.gen_gather.argtypes = [p, p, u64, u32, p]
        L.gen_poisson_arrivals.argtypes = [u64, ctypes.c_double, p, u64]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def xs64(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    lib().gen_xs64(seed, _ptr(out), n)
    return out


def words(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    lib().gen_words(seed, _ptr(out), n)
    return out


def permutation(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    lib().gen_permutation(seed, _ptr(out), n)
    return out


@dataclasses.dataclass
class Model:
    """A synthetic guarded-interleaving model.

    trans[p, l, k] = (target, guard_var, guard_val, eff_var, eff_val), with
    NONE (0xFFFFFFFF) in guard_var / eff_var meaning "no guard" / "no effect".
    init has W = P + S words.  cap is the level-prefix state cap (0 = none).
    """
    P: int
    L: int
    S: int
    D: int
    K: int
    trans: np.ndarray
    init: np.ndarray
    cap: int = 0
    name: str = ""
    seed: int = 0

    @property
    def W(self) -> int:
        return self.P + self.S

    def describe(self) -> dict:
        return dict(name=self.name, seed=self.seed, P=self.P, L=self.L, S=self.S,
                    D=self.D, K=self.K, W=self.W, cap=self.cap)


def guarded_model(seed: int, P: int, L: int, S: int, D: int, K: int = 3,
                  cap: int = 0, name: str = "") -> Model:
    trans = np.empty((P, L, K, 5), dtype=np.uint32)
    rc = lib().gen_guarded_model(seed, P, L, S, D, K, _ptr(trans))
    if rc != 0:
        raise ValueError("bad model sizes")
    init = np.zeros(P + S, dtype=np.uint32)
    return Model(P, L, S, D, K, trans, init, cap, name or f"G({seed:#x},{P},{L},{S},{D},{K})", seed)


def cyclic_model(N: int, L: int, cap: int = 0) -> Model:
    """N independent cyclic L-state processes (step l -> (l+1) mod L)."""
    trans = np.empty((N, L, 1, 5), dtype=np.uint32)
    if lib().gen_cyclic_model(N, L, _ptr(trans)) != 0:
        raise ValueError("bad model sizes")
    init = np.zeros(N, dtype=np.uint32)
    return Model(N, L, 0, 1, 1, trans, init, cap, f"cyclic({N},{L})", 0)


def dup_stream(seed: int, n_distinct: int, W: int, copies: int = 2):
    """(rows [n_distinct, W] u32, order [n_distinct*copies] u32)."""
    rows = np.empty((n_distinct, W), dtype=np.uint32)
    order = np.empty(n_distinct * copies, dtype=np.uint32)
    lib().gen_dup_stream(seed, n_distinct, W, copies, _ptr(rows), _ptr(order))
    return rows, order


def gather(rows: np.ndarray, order: np.ndarray) -> np.ndarray:
    W = rows.shape[1]
    out = np.empty((order.shape[0], W), dtype=np.uint32)
    lib().gen_gather(_ptr(rows), _ptr(order), order.shape[0], W, _ptr(out))
    return out


def poisson_arrivals(seed: int, lam: float, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().gen_poisson_arrivals(seed, lam, _ptr(out), n)
    return out


# ---------------------------------------------------------------------------
# Workload recipes (synthetic stand-ins for the paper's BEEM benchmark set).

#: Raw find-or-put stream: 2^25 distinct 16-word rows, each occurring twice.
STREAM_SEED = 0x2545F4914F6CDD1D
STREAM_W = 16
STREAM_DISTINCT = 1 << 25
STREAM_TABLE_SLOTS = 1 << 28

#: Large synthetic model: 12 processes x 16 local states, 4 shared vars.
BIG_P, BIG_L, BIG_S, BIG_K = 12, 16, 4, 3
BIG_CAP = 1 << 27
BIG_TABLE_SLOTS = 1 << 28

_MANIFEST_DIR = os.path.join(_HERE, "manifests")


def tiny_cyclic() -> Model:
    """4 cyclic 8-state processes, 4 words, 8^4 = 4096 reachable states."""
    return cyclic_model(4, 8)


def stream_workload(n_distinct: int = STREAM_DISTINCT, W: int = STREAM_W,
                    seed: int = STREAM_SEED, copies: int = 2):
    """rows, order for the duplicate stream (materialise with gather())."""
    return dup_stream(seed, n_distinct, W, copies)


def _load_manifest(name: str) -> dict:
    with open(os.path.join(_MANIFEST_DIR, name)) as f:
        return json.load(f)


def big_model(cap: int = BIG_CAP) -> Model:
    """The 12x16 model whose seed (recorded in manifests/big_model.json) was
    chosen so that its state space exceeds the 2^27 cap."""
    m = _load_manifest("big_model.json")
    return guarded_model(int(m["seed"], 0), BIG_P, BIG_L, BIG_S, m["D"], BIG_K,
                         cap=cap, name="big12x16")


#: Uncapped model explored to exhaustion (no cap, so the exploration without
#: levels and the BFS define the same result): 8 processes x 6 local states,
#: 4 shared variables of domain 4, 2 transitions per local state; the seed
#: was picked from a scan of seeds for a full state space of a few 10^7
#: states (32 518 299 states in 104 BFS levels).
WIDE_SEED, WIDE_P, WIDE_L, WIDE_S, WIDE_D, WIDE_K = 78, 8, 6, 4, 4, 2
WIDE_TABLE_SLOTS = 1 << 26


def wide_model() -> Model:
    return guarded_model(WIDE_SEED, WIDE_P, WIDE_L, WIDE_S, WIDE_D, WIDE_K, cap=0, name="wide8x6")


def chain_model(n: int = 20000) -> Model:
    """One process stepping through n local states: n BFS levels of one
    state each (the narrowest state space, where level barriers cost most)."""
    return cyclic_model(1, n)


def batch_models() -> list[Model]:
    """The 64-model mix (manifests/batch_models.json): 2-16 processes,
    4-32 local states, state width 4-32, 10^3-10^6 reachable states each."""
    m = _load_manifest("batch_models.json")
    out = []
    for e in m["models"]:
        out.append(guarded_model(int(e["seed"], 0), e["P"], e["L"], e["S"], e["D"],
                                 e.get("K", 3), cap=0, name=e.get("name", "")))
    return out


def draw_batch_params(master_seed: int, trial: int) -> dict:
    """Parameters of candidate model `trial` of the batch mix.

    P in [2,16], S in [2,16] with 4 <= P+S <= 32, L in [4,32], D in [2,16];
    the model seed is a further xorshift64 output.  Deterministic in
    (master_seed, trial)."""
    x = xs64(master_seed ^ (0x9E3779B97F4A7C15 * (trial + 1) & 0xFFFFFFFFFFFFFFFF), 8)
    P = 2 + int(x[0] % 15)
    S = 2 + int(x[1] % 15)
    L = 4 + int(x[2] % 29)
    D = 2 + int(x[3] % 15)
    seed = int(x[4]) or 1
    while P + S > 32:
        S -= 1
    return dict(P=P, L=L, S=S, D=D, K=3, seed=seed)
