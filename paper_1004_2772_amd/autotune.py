"""Autotuner of the table shape: line width (8/16/32 slots), probe sequence
across lines (double hashing / linear / quadratic) and GPU lanes per
operation, for find-or-put and for BFS expansion.

    python -m paper_1004_2772_amd.autotune [--out PATH] [--widths 4,8,16,32]
        [--log2-caps 20,24,28] [--reps 3] [--no-batch]

For every (state width W, table size 2^c) it times, on the current GPU and
through the library's C-ABI:
  * the batched find-or-put of a stream of 2^c/8 distinct seeded random
    W-word vectors (gen.dup_stream), each occurring twice in shuffled order
    (load factor 1/8), one call into an empty table, for every line width x
    probe x lanes;
  * a level-synchronous BFS of a synthetic guarded model of width W capped
    at 2^c/4 states, for every line width x probe x lanes;
and for the batch kind, the 64-model mix explored in one persistent launch.
Per key it keeps the line width and probe whose times, each divided by the
best time of its workload, sum lowest (double hashing preferred within 3 %),
and with them the fastest lanes for each workload.  Every shape gives
identical results; only speed differs.

The file it writes is read by lhs_tune_load (format "lhs-tune-1"); the
measured times are kept in each entry.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

from . import (PROBES, TUNE_PATH_DEFAULT, LhsError, Table, config, reach_explore,
               reach_explore_batch)

LINES = (8, 16, 32)
PROBE_NAMES = tuple(PROBES)
TPS = (1, 4, 8, 16)
SEED = 0x7E57


def log(msg):
    print(f"[autotune {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _key(ls, probe, tps):
    return f"{ls}/{probe}/{tps}"


def _timed(fn, reps):
    """Median device time (ms) of fn over `reps` runs after one warm-up; fn
    returns its own time in ms."""
    fn()
    return statistics.median(fn() for _ in range(reps))


def time_stream(W: int, log2cap: int, reps: int) -> dict:
    import torch

    import gen
    cap = 1 << log2cap
    n_distinct = cap // 8
    rows, order = gen.dup_stream(SEED + 97 * W + log2cap, n_distinct, W)
    states = torch.from_numpy(gen.gather(rows, order).view(np.int32)).cuda()
    del rows, order
    n = states.shape[0]
    seen = torch.empty(n, dtype=torch.uint8, device="cuda")
    idx = torch.empty(n, dtype=torch.int32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for ls in LINES:
        for probe in PROBE_NAMES:
            with Table(cap, W, config(ls, probe)) as t:
                for tps in TPS:
                    t.set_threads_per_state(tps)

                    def run():
                        t.clear()
                        e0.record()
                        t.find_or_put(states, seen, idx)
                        e1.record()
                        e1.synchronize()
                        return e0.elapsed_time(e1)

                    out[_key(ls, probe, tps)] = round(_timed(run, reps), 4)
                    t.check()
                    new = int((seen == 0).sum().item())
                    if new != n_distinct:
                        raise RuntimeError(f"stream W={W} 2^{log2cap} {_key(ls, probe, tps)}: "
                                           f"{new} new rows, expected {n_distinct}")
    del states, seen, idx
    torch.cuda.empty_cache()
    return out


def bfs_model(W: int, state_cap: int):
    """A guarded synthetic model of width W whose BFS reaches the cap (the
    first of a fixed list of seeds that does)."""
    import gen
    P = max(1, (3 * W) // 4)
    S = W - P
    L = 1024 if W <= 4 else (64 if W <= 8 else 16)
    for seed in range(1, 40):
        m = gen.guarded_model(seed, P, L, S, 8, 3, cap=state_cap, name=f"tune{W}")
        r = reach_explore(m, capacity=_bfs_capacity(state_cap))
        if r.capped:
            return m, r
    return m, r


def _bfs_capacity(state_cap):
    return 1 << max(12, (4 * state_cap).bit_length() - 1)


def time_bfs(W: int, log2cap: int, reps: int) -> tuple[dict, dict]:
    state_cap = (1 << log2cap) // 4
    m, ref = bfs_model(W, state_cap)
    desc = {"P": m.P, "L": m.L, "S": m.S, "K": m.K, "seed": m.seed, "state_cap": state_cap,
            "states": ref.total, "levels": ref.n_levels, "edges": ref.edges}
    out = {}
    for ls in LINES:
        for probe in PROBE_NAMES:
            with Table(1 << log2cap, W, config(ls, probe)) as t:
                for tps in TPS:
                    t.set_threads_per_state(tps)

                    def run():
                        r = reach_explore(m, table=t)
                        if (r.total, r.edges, r.level_counts) != (ref.total, ref.edges, ref.level_counts):
                            raise RuntimeError(f"bfs W={W} {_key(ls, probe, tps)} differs from the "
                                               f"default shape's result")
                        return r.gpu_ms

                    out[_key(ls, probe, tps)] = round(_timed(run, reps), 4)
    return out, desc


def time_batch(reps: int) -> tuple[dict, dict]:
    import gen
    models = gen.batch_models()
    ref = None
    out = {}
    for ls in LINES:
        for probe in PROBE_NAMES:
            tables = [Table(1 << 21, m.W, config(ls, probe)) for m in models]
            try:
                for tps in TPS:
                    for t in tables:
                        t.set_threads_per_state(tps)

                    def run():
                        nonlocal ref
                        rs = reach_explore_batch(models, tables=tables)
                        got = [(r.total, r.edges) for r in rs]
                        if ref is None:
                            ref = got
                        elif got != ref:
                            raise RuntimeError(f"batch {_key(ls, probe, tps)} results differ")
                        return rs[0].gpu_ms

                    out[_key(ls, probe, tps)] = round(_timed(run, reps), 4)
            finally:
                for t in tables:
                    t.close()
    return out, {"models": len(models), "states": sum(r[0] for r in ref)}


# Probe sequences in order of preference when their times are within
# TOLERANCE of each other: double hashing keeps probe chains short as the
# table fills (linear probing clusters), which the timed workloads, at load
# factor 1/8, do not show.
PROBE_PREFERENCE = ("double", "quadratic", "linear")
TOLERANCE = 0.03


def choose(times_a: dict, times_b: dict | None):
    """(line_slots, probe, best tps for a, best tps for b) minimising the sum of
    each workload's best time at that (line, probe) over its overall best;
    among (line, probe) pairs within TOLERANCE of the lowest sum, the
    preferred probe sequence wins, then the lower sum."""
    best_a = min(times_a.values())
    best_b = min(times_b.values()) if times_b else None
    scored = []
    for ls in LINES:
        for probe in PROBE_NAMES:
            ta = {tps: times_a[_key(ls, probe, tps)] for tps in TPS}
            score = min(ta.values()) / best_a
            tb = None
            if times_b:
                tb = {tps: times_b[_key(ls, probe, tps)] for tps in TPS}
                score += min(tb.values()) / best_b
            scored.append((score, ls, probe, min(ta, key=ta.get), min(tb, key=tb.get) if tb else None))
    low = min(x[0] for x in scored)
    near = [x for x in scored if x[0] <= low * (1 + TOLERANCE)]
    pick = min(near, key=lambda x: (PROBE_PREFERENCE.index(x[2]), x[0]))
    return pick[1:], pick[0]


def reselect(path: str):
    """Apply the selection rule again to the times recorded in a tuning file."""
    with open(path) as f:
        doc = json.load(f)
    for e in doc["entries"]:
        if e["kind"] == "table":
            (ls, probe, tf, te), score = choose(e["stream_ms"], e["bfs_ms"])
        else:
            (ls, probe, te, _), score = choose(e["batch_ms"], None)
            tf = 0
        e.update(line_slots=ls, probe=probe, tps_find_or_put=tf, tps_expand=te, score=round(score, 4))
    doc["selection"] = f"probe preference {list(PROBE_PREFERENCE)} within {TOLERANCE:.0%}"
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1)
    os.replace(tmp, path)
    return doc


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TUNE_PATH_DEFAULT)
    ap.add_argument("--widths", default="4,8,16,32")
    ap.add_argument("--log2-caps", default="20,24,28")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--reselect", metavar="PATH",
                    help="only re-apply the selection rule to the times recorded in PATH")
    a = ap.parse_args(argv)
    if a.reselect:
        return reselect(a.reselect)

    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the autotuner times kernels on a GPU")
    props = torch.cuda.get_device_properties(0)
    arch = props.gcnArchName.split(":")[0]
    entries = []
    t_start = time.time()
    for W in [int(x) for x in a.widths.split(",") if x]:
        for lc in [int(x) for x in a.log2_caps.split(",") if x]:
            log(f"W={W} table 2^{lc}: find-or-put stream")
            ts = time_stream(W, lc, a.reps)
            log(f"W={W} table 2^{lc}: BFS")
            tb, desc = time_bfs(W, lc, a.reps)
            (ls, probe, tf, te), score = choose(ts, tb)
            log(f"W={W} 2^{lc}: line_slots={ls} probe={probe} tps_find_or_put={tf} tps_expand={te} "
                f"(stream {ts[_key(ls, probe, tf)]:.3f} ms, best {min(ts.values()):.3f}; "
                f"bfs {tb[_key(ls, probe, te)]:.3f} ms, best {min(tb.values()):.3f})")
            entries.append({"kind": "table", "W": W, "log2_capacity": lc, "line_slots": ls,
                            "probe": probe, "tps_find_or_put": tf, "tps_expand": te,
                            "score": round(score, 4), "stream_ms": ts, "bfs_ms": tb,
                            "bfs_model": desc})
    if not a.no_batch:
        log("batch: 64-model mix, one persistent launch")
        tb, desc = time_batch(a.reps)
        (ls, probe, te, _), score = choose(tb, None)
        log(f"batch: line_slots={ls} probe={probe} tps_expand={te} ({tb[_key(ls, probe, te)]:.3f} ms, "
            f"default 16/double/1: {tb[_key(16, 'double', 1)]:.3f} ms)")
        entries.append({"kind": "batch", "W": 32, "log2_capacity": 21, "line_slots": ls, "probe": probe,
                        "tps_find_or_put": 0, "tps_expand": te, "score": round(score, 4),
                        "batch_ms": tb, "batch_workload": desc})
    doc = {"format": "lhs-tune-1", "device": arch, "cus": props.multi_processor_count,
           "generator": "python -m paper_1004_2772_amd.autotune " + " ".join(argv or sys.argv[1:]),
           "seconds": round(time.time() - t_start, 1),
           "selection": f"probe preference {list(PROBE_PREFERENCE)} within {TOLERANCE:.0%}",
           "entries": entries}
    tmp = a.out + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1)
    os.replace(tmp, a.out)
    log(f"wrote {a.out} ({len(entries)} entries, {doc['seconds']} s)")
    return doc


if __name__ == "__main__":
    try:
        main()
    except LhsError as e:
        sys.exit(f"autotune failed: {e}")
