#!/usr/bin/env python3
"""Benchmark of the lockless find-or-put table on one MI355X.

Headline step (the raw find-or-put workload): a stream of 2^26 state vectors
of 16 x uint32, 2^25 distinct rows each occurring twice in a seeded shuffled
order (50 % exact duplicates), inserted into an empty 2^28-slot table with one
batched find-or-put call.  A step = clear the table + the find-or-put pass;
the value is find-or-put operations per second over the timed steps, with the
inputs already resident in HBM.

Extra legs in the same JSON line:
  roofline     : the find-or-put kernel's algorithmic bytes per launch (one
                 128-byte slot line and one 64-byte row per operation, 192 B)
                 over its average duration (HIP events on the launch stream),
                 against the 8 TB/s HBM peak and against the measured random
                 128-byte line ceiling; hardware traffic from committed
                 rocprofv3 counter summaries when they match the kernel source.
  probes       : measured ceilings: random line reads of 64/128/256 bytes
                 (cooperative lanes, and 128 B by one lane) and random 64-bit
                 CAS throughput, random slot stores, row stores and row loads;
                 the find-or-put's algorithmic GB/s over the line ceiling at
                 its table's line width, and its launch time over the sum of
                 its accesses priced at the probes' rates.
  bfs          : level-synchronous BFS of the 12-process x 16-local synthetic
                 model capped at 2^27 states (states/s, edges/s); the same BFS
                 with one find-or-put per successor (merging of equal
                 successors of a pass off), and the share of edges merged.
  batch        : the 64-model mix (2-16 processes, widths 4-32, 10^3-10^6
                 states each) explored in one persistent launch, in one launch
                 per step, and one model at a time, on the same tables.
  serve        : Poisson arrivals (200/s for 60 s, the first 5 s excluded) of
                 queries drawn uniformly from the mix, served with continuous
                 batching by the persistent launch and, for comparison, one
                 query at a time (--serve-rounds adds host rounds of level
                 steps); p50/p99 latency from scheduled arrival, states per
                 second of server work; and a burst of queries submitted at
                 once, where the GPU and not the arrivals bounds the states
                 per second.
  cpu_baseline : the CPU oracle (sequential find-or-put) timed on a bounded
                 prefix of the same stream, one host thread; bfs.cpu_baseline
                 and batch.cpu_baseline time the oracle's BFS on the model
                 capped at 2^22 states and over the 64-model mix.
  cpu_lockless : the paper's lockless table and level-synchronous BFS on all
                 host cores (cpu_table/), on the same stream and on the model
                 capped at 2^22 states.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "states/sec and find-or-put ops/sec at 1 GPU; % of HBM random-access roofline"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
FOP_SOURCES = ["paper_1004_2772_amd/csrc/lhs_device.h", "paper_1004_2772_amd/csrc/lhs_table.hip"]


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def source_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def fop_bytes_per_op(W, line_slots=16):
    """The build's own count of one find-or-put's bytes at its table's line
    width: input row, one line of 8-byte slots, one row of data (written if
    new, compared if seen), seen byte + index."""
    return 4 * W + 8 * line_slots + 4 * W + 1 + 4


def spec_bytes_per_op(W):
    """Random bytes one find-or-put must move by the method: one 128-byte
    line of slots (about one line per operation at low fill) and one row of
    data written (new) or read (seen), in 64-byte pieces: 192 B at W = 16.
    Sequential input and output are counted apart."""
    return 128 + 64 * ((4 * W + 63) // 64)


def load_traffic(kernel, workload, n_launch_ops):
    """Hardware bytes per launch from a committed counter summary, or None
    if it is missing or was taken on different kernel source."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha") != source_sha(FOP_SOURCES) or t.get("ops_per_launch") != n_launch_ops:
        return None, t
    return int(t["fetch_bytes"] + t["write_bytes"]), t


def load_atomics(kernel, workload, n_launch_ops):
    """Atomic requests per launch (rocprofv3 TCC counters) of the kernel and
    of the random-CAS probe, or None if missing or taken on other sources."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_atomics.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha") != source_sha(FOP_SOURCES) or t.get("ops_per_launch") != n_launch_ops:
        return None
    return t


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--distinct", type=int, default=1 << 25, help="distinct rows (each twice)")
    ap.add_argument("--table-log2", type=int, default=28)
    ap.add_argument("--batch", type=int, default=0, help="rows per call (0 = whole stream)")
    ap.add_argument("--no-bfs", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-cpu-lockless", action="store_true",
                    help="skip the multi-core CPU lockless-table leg")
    ap.add_argument("--no-probes", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-async", action="store_true", help="skip the exploration-without-levels leg")
    ap.add_argument("--no-chain", action="store_true",
                    help="in that leg, skip the chain of one-state levels (tens of thousands of launches)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="query arrivals per second")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-warmup", type=float, default=5.0, help="seconds excluded from latency stats")
    ap.add_argument("--serve-rounds", action="store_true",
                    help="also serve the stream with host rounds of level steps instead of the persistent launch")
    ap.add_argument("--serve-burst", type=int, default=1000,
                    help="queries submitted at once for the saturated serving point (0 = skip)")
    ap.add_argument("--calib-copy", action="store_true", help="also run the copy probe (counter calibration)")
    ap.add_argument("--bfs-cap", type=int, default=1 << 27)
    ap.add_argument("--cpu-sample", type=int, default=1 << 25)
    ap.add_argument("--tps", type=int, default=0, help="lanes per operation (0 = library default)")
    ap.add_argument("--sweep-tps", action="store_true", help="also time every threads-per-state value")
    ap.add_argument("--no-tune", action="store_true",
                    help="ignore the package's tuning table (default table shapes)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_1004_2772_amd as lhs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    lhs.lib()   # fails loudly if the HIP library is missing
    n_tuned = 0 if args.no_tune else lhs.tune_load_default()
    log(f"tuning table: {n_tuned} entries loaded")

    W = gen.STREAM_W
    n_distinct = args.distinct
    n = 2 * n_distinct
    batch = args.batch or n
    log(f"generating stream: {n} rows of {W} words ({n_distinct} distinct)")
    rows, order = gen.stream_workload(n_distinct=n_distinct, W=W)
    rows_d = torch.from_numpy(rows.view(np.int32)).to(dev)
    order_d = torch.from_numpy(order.astype(np.int64)).to(dev)
    states_d = rows_d.index_select(0, order_d)          # input resident in HBM
    del rows_d, order_d
    seen_d = torch.empty(n, dtype=torch.uint8, device=dev)
    idx_d = torch.empty(n, dtype=torch.int32, device=dev)
    table = lhs.Table(1 << args.table_log2, W)
    if args.tps:
        table.set_threads_per_state(args.tps)
    torch.cuda.synchronize()

    kernel_events = []

    def step(record):
        table.clear()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for lo in range(0, n, batch):
            hi = min(n, lo + batch)
            table.find_or_put(states_d[lo:hi], seen_d[lo:hi], idx_d[lo:hi])
        e1.record(stream)
        if record:
            kernel_events.append((e0, e1))

    for i in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    table.check()
    log(f"warmup done ({args.warmup} steps)")

    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.time()
    t0.record(stream)
    for i in range(args.steps):
        step(True)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - wall0
    total_ms = t0.elapsed_time(t1)
    ms_per_step = total_ms / args.steps
    kern_ms = sum(a.elapsed_time(b) for a, b in kernel_events) / len(kernel_events)
    n_launch = (n + batch - 1) // batch
    launch_ms = kern_ms / n_launch
    table.check()
    new = int((seen_d == 0).sum().item())
    stored = table.count()
    ok = new == n_distinct and stored == n_distinct and int((seen_d > 1).sum().item()) == 0
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, find-or-put {kern_ms:.3f} ms, "
        f"new={new} stored={stored} ok={ok}")
    info = table.info()

    def time_fop(tps, reps=3):
        table.set_threads_per_state(tps)
        ts = []
        for _ in range(reps):
            table.clear()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            table.find_or_put(states_d, seen_d, idx_d)
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        table.check()
        return sorted(ts)[len(ts) // 2]

    sweep = {}
    if args.sweep_tps:
        for tps in (1, 4, 8, 16):
            ms = time_fop(tps)
            sweep[str(tps)] = {"fop_ms": round(ms, 3), "fop_Gops": round(n / ms / 1e6, 3)}
            log(f"tps={tps}: find-or-put {ms:.3f} ms")
        table.set_threads_per_state(0)

    ops_per_s = n / (ms_per_step / 1e3)
    bpo = spec_bytes_per_op(W)
    own_bpo = fop_bytes_per_op(W, info["line_slots"])
    launch_ops = min(batch, n)
    achieved = bpo * launch_ops / (launch_ms / 1e3) / 1e9
    traffic, tinfo = load_traffic("k_find_or_put", "stream2p26", launch_ops)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_find_or_put", "avg_launch_ms": round(launch_ms, 4),
                "algorithmic_bytes_per_op": bpo, "ops_per_launch": launch_ops,
                "own_accounting": {"bytes_per_op": own_bpo,
                                   "what": f"input row + one {8 * info['line_slots']}-byte line (the "
                                           f"table's) + one row + seen byte and index",
                                   "GBs": round(own_bpo * launch_ops / (launch_ms / 1e3) / 1e9, 1)}}
    if tinfo is not None:
        roofline["traffic_source"] = os.path.basename(tinfo.get("summary", ""))
        if traffic:
            roofline["traffic_over_algorithmic"] = round(traffic / (bpo * launch_ops), 3)
            roofline["hbm_traffic_GBs"] = round(traffic / (launch_ms / 1e3) / 1e9, 1)
            roofline["hbm_traffic_frac"] = round(traffic / (launch_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)

    props = torch.cuda.get_device_properties(0)
    cpu_name = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_name = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    out = {
        "metric": METRIC, "value": round(ops_per_s, 1), "unit": "find-or-put ops/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"find-or-put stream: {n} rows of {W} x uint32 ({n_distinct} distinct, "
                               f"each twice, shuffled), table 2^{args.table_log2} slots, "
                               f"{n_launch} call(s) per step",
                   "ops": n, "distinct": n_distinct, "state_words": W,
                   "table_slots": 1 << args.table_log2, "batch": launch_ops,
                   "load_factor": round(n_distinct / (1 << args.table_log2), 4)},
        "roofline": roofline,
        "checks": {"new_equals_distinct": ok, "wait_hits": info["wait_hits"],
                   "cas_failures": info["cas_failures"]},
        "table_shape": {"tuning_entries": n_tuned, "stream_table": table.config(),
                        "tps_in_effect": [info["tps_find_or_put"], info["tps_expand"]]},
        "wall_s_timed": round(wall, 3),
        "host": {"gpu": props.name, "arch": props.gcnArchName, "cus": props.multi_processor_count,
                 "hbm_gib": round(props.total_memory / 2**30, 1), "cpu": cpu_name,
                 "nproc": os.cpu_count()},
    }

    if not args.no_probes:
        sink = torch.zeros(1, dtype=torch.int64, device=dev)
        buf = torch.empty(1 << 32, dtype=torch.int32, device=dev)     # 16 GiB
        probes = {}
        for lb, lanes in ((128, 1), (64, 4), (128, 8), (256, 16)):
            reads = (1 << 34) // lb // 8          # 2 GiB of lines per probe
            lhs.probe_random_lines(buf, lb, lanes, reads, 1, sink)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lhs.probe_random_lines(buf, lb, lanes, reads, 2, sink)
            b.record(stream)
            torch.cuda.synchronize()
            probes[f"random_{lb}B_lines_{lanes}lane_GBs"] = round(reads * lb / (a.elapsed_time(b) / 1e3) / 1e9, 1)
        for form in ("slot_store", "row_store", "row_load"):
            ops = 1 << 27
            lhs.probe_random_access(buf, form, ops, 5, sink)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lhs.probe_random_access(buf, form, ops, 6, sink)
            b.record(stream)
            torch.cuda.synchronize()
            probes[f"random_{form}_Gops"] = round(ops / (a.elapsed_time(b) / 1e3) / 1e9, 3)
        del buf
        slots = torch.zeros(1 << 28, dtype=torch.int64, device=dev)
        ops = 1 << 26
        lhs.probe_random_cas(slots, ops, 3, sink)
        slots.zero_()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        lhs.probe_random_cas(slots, ops, 4, sink)
        b.record(stream)
        torch.cuda.synchronize()
        probes["random_cas64_Gops"] = round(ops / (a.elapsed_time(b) / 1e3) / 1e9, 3)
        del slots
        lb = 8 * info["line_slots"]
        ceiling = probes[f"random_{lb}B_lines_{lb // 16}lane_GBs"]
        # the primary denominator: random 128-byte lines read by 8 lanes each
        line128 = probes["random_128B_lines_8lane_GBs"]
        roofline["random_128B_line_GBs"] = line128
        roofline["frac_of_random_128B_line"] = round(achieved / line128, 4)
        roofline["meets_40pct_of_random_128B_line"] = achieved / line128 >= 0.40
        probes["fop_own_bytes_frac_of_table_line_ceiling"] = round(
            roofline["own_accounting"]["GBs"] / ceiling, 4)
        probes["fop_table_line_ceiling"] = f"random_{lb}B_lines_{lb // 16}lane_GBs"
        # slot CAS issued by the find-or-put launch (one per insert plus the
        # retries) against the random 64-bit CAS rate of the same GPU
        cas = n_distinct + info["cas_failures"]
        # the whole access mix of the launch priced at the probes' rates, as
        # if served one after another: per operation one slot line read (at
        # 1/8 fill an operation examines 1.00 lines), per lookup one row
        # load, per insert one row store and one DONE store, and every CAS
        line_rate = probes[f"random_{lb}B_lines_{lb // 16}lane_GBs"] * 1e9 / lb
        mix = {"line_reads": n / line_rate,
               "row_loads": (n - n_distinct) / (probes["random_row_load_Gops"] * 1e9),
               "cas": cas / (probes["random_cas64_Gops"] * 1e9),
               "row_stores": n_distinct / (probes["random_row_store_Gops"] * 1e9),
               "slot_stores": n_distinct / (probes["random_slot_store_Gops"] * 1e9)}
        mix_s = sum(mix.values())
        probes["fop_access_mix_ms"] = {k: round(v * 1e3, 3) for k, v in mix.items()}
        probes["fop_access_mix_sum_ms"] = round(mix_s * 1e3, 3)
        probes["fop_launch_over_access_mix_sum"] = round(launch_ms / 1e3 / mix_s, 4) if n_launch == 1 else None
        cas_per_s = cas / (launch_ms / 1e3) if n_launch == 1 else None
        probes["fop_cas_per_s"] = round(cas_per_s, 1) if cas_per_s else None
        probes["fop_cas_frac_of_random_cas"] = (round(cas_per_s / 1e9 / probes["random_cas64_Gops"], 4)
                                                if cas_per_s else None)
        # the same from rocprofv3: L2 atomic requests per launch (committed
        # counter summary) over this run's launch times
        at = load_atomics("k_find_or_put", "stream2p26", launch_ops)
        if at is not None and n_launch == 1:
            probe_s = (1 << 26) / (probes["random_cas64_Gops"] * 1e9)
            fop_rate = at["l2_atomics_per_launch"] / (launch_ms / 1e3)
            probe_rate = at["probe_l2_atomics_per_launch"] / probe_s
            out["atomics"] = {"source": "k_find_or_put_stream2p26_atomics.json (rocprofv3 TCC_ATOMIC_sum)",
                              "fop_l2_atomics_per_op": round(at["l2_atomics_per_op"], 4),
                              "fop_l2_atomics_per_s": round(fop_rate, 1),
                              "probe_l2_atomics_per_s": round(probe_rate, 1),
                              "frac_of_random_cas": round(fop_rate / probe_rate, 4)}
        out["probes"] = probes
        log(f"probes: {probes}")

    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.int32, device=dev)        # 1 GiB
        dst = torch.empty_like(src)
        lhs.probe_copy(dst, src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = src.numel() * 4
        del src, dst

    if not args.no_bfs:
        m = gen.big_model(cap=args.bfs_cap)
        runs = []
        res = None
        for i in range(1 + max(1, min(args.steps, 3))):
            w0 = time.time()
            res = lhs.reach_explore(m, table=table)
            if i:
                runs.append((res.gpu_ms, time.time() - w0))
            log(f"bfs run {i}: {res.total} states, {res.n_levels} levels, {res.gpu_ms:.1f} ms")
        gms = sorted(r[0] for r in runs)[len(runs) // 2]
        bfs = {"workload": f"BFS of G(seed={m.seed}, P=12, L=16, S=4, D={m.D}, K=3), "
                           f"level-prefix cap {args.bfs_cap}, table 2^{args.table_log2}",
               "states": res.total, "levels": res.n_levels, "edges": res.edges,
               "deadlocks": res.deadlocks, "capped": res.capped, "median_ms": round(gms, 2),
               "states_per_s": round(res.total / (gms / 1e3), 1),
               "edges_per_s": round(res.edges / (gms / 1e3), 1), "wait_hits": res.wait_hits}
        # algorithmic bytes of the exploration: per edge one 128-byte slot
        # line and one row (as for find-or-put), per expanded state its row
        # and frontier index, per new state its frontier entry
        expanded = res.total - (res.level_counts[-1] if res.capped else 0)
        per_edge, per_exp = spec_bytes_per_op(m.W), 4 * m.W + 4
        bfs_bytes = res.edges * per_edge + expanded * per_exp + (res.total - 1) * 4
        bfs_gbs = bfs_bytes / (gms / 1e3) / 1e9
        bfs["roofline"] = {"bound": "hbm", "kernel": "k_expand (the whole exploration, its first levels in "
                                                     "k_batch_persistent)",
                           "bytes_per_edge": per_edge, "bytes_per_expanded_state": per_exp,
                           "bytes_per_new_state": 4, "algorithmic_bytes": bfs_bytes,
                           "achieved": round(bfs_gbs, 1), "peak": 8000.0, "unit": "GB/s",
                           "frac": round(bfs_gbs / 8000.0, 4)}
        tpath = os.path.join(ROOT, "profiles", "k_expand_bfs2p27_traffic.json")
        if os.path.exists(tpath) and args.bfs_cap == 1 << 27:
            with open(tpath) as f:
                tr = json.load(f)
            bfs["roofline"]["traffic_bytes_per_edge"] = round(tr["fetch_bytes_per_edge"] + tr["write_bytes_per_edge"], 1)
            bfs["roofline"]["traffic_source"] = "k_expand_bfs2p27_traffic.json (rocprofv3 FETCH_SIZE + WRITE_SIZE)"
        golden = os.path.join(ROOT, "tests", "golden", "big_model.json")
        if os.path.exists(golden) and args.bfs_cap == 1 << 27:
            with open(golden) as f:
                g = json.load(f)
            bfs["matches_oracle_counts"] = (g["level_counts"] == res.level_counts and
                                            g["edges"] == res.edges and g["deadlocks"] == res.deadlocks)
        gruns = []
        for i in range(1 + max(1, min(args.steps, 3))):
            rg = lhs.reach_explore(m, table=table, flags=lhs.REACH_F_GRAPH)
            if i:
                gruns.append(rg.gpu_ms)
            log(f"bfs graph run {i}: {rg.total} states, {rg.n_levels} levels, {rg.gpu_ms:.1f} ms")
        gg = sorted(gruns)[len(gruns) // 2]
        bfs["graph_levels"] = {"median_ms": round(gg, 2), "states_per_s": round(rg.total / (gg / 1e3), 1),
                               "same_result": (rg.total, rg.level_counts, rg.edges) ==
                                              (res.total, res.level_counts, res.edges)}
        # equal successors of a pass merged (the default) against one
        # find-or-put per successor, and the share of edges merged
        table.set_merge(lhs.MERGE_OFF)
        oruns = []
        for i in range(1 + max(1, min(args.steps, 3))):
            ro = lhs.reach_explore(m, table=table)
            if i:
                oruns.append(ro.gpu_ms)
        table.set_merge(lhs.MERGE_ON)
        table.set_counters(lhs.COUNT_MERGED)
        rc = lhs.reach_explore(m, table=table)
        merged = table.info()["merged"]
        table.set_counters(0)
        om = sorted(oruns)[len(oruns) // 2]
        bfs["merge"] = {"merged_edges": merged, "merged_per_edge": round(merged / rc.edges, 4),
                        "merge_off_median_ms": round(om, 2), "merge_off_wait_hits": ro.wait_hits,
                        "speedup_of_merging": round(om / gms, 3),
                        "same_result": (ro.total, ro.level_counts, ro.edges, ro.deadlocks) ==
                                       (res.total, res.level_counts, res.edges, res.deadlocks) ==
                                       (rc.total, rc.level_counts, rc.edges, rc.deadlocks)}
        log(f"bfs merging off: {om:.1f} ms; merged {merged} of {rc.edges} edges")
        # the paper's speedup S = T_1 / T_N and efficiency E = S / N over N
        # workers (one workgroup of 256 lanes each), on a 2^22-state prefix
        # of the same model
        mw = gen.big_model(cap=1 << 22)
        with lhs.Table(1 << 24, mw.W) as tw:
            ws = {}
            for nw in (1, 1024):
                tw.set_workers(nw)
                rw = [lhs.reach_explore(mw, table=tw) for _ in range(3)]
                ws[nw] = (sorted(r.gpu_ms for r in rw[1:])[0], rw[-1])
        s_w = ws[1][0] / ws[1024][0]
        bfs["workers_speedup"] = {"workload": f"BFS of the same model capped at 2^22 states ({ws[1][1].total} states)",
                                  "ms_1_workgroup": round(ws[1][0], 2), "ms_1024_workgroups": round(ws[1024][0], 2),
                                  "speedup_S": round(s_w, 1), "efficiency_E": round(s_w / 1024, 3),
                                  "same_result": ws[1][1].level_counts == ws[1024][1].level_counts}
        log(f"bfs workers: 1 workgroup {ws[1][0]:.1f} ms, 1024 workgroups {ws[1024][0]:.2f} ms, S = {s_w:.1f}")
        if args.sweep_tps:
            for tps in (1, 4, 8, 16):
                table.set_threads_per_state(tps)
                r = lhs.reach_explore(m, table=table)
                sweep[str(tps)]["bfs_ms"] = round(r.gpu_ms, 2)
                log(f"tps={tps}: bfs {r.gpu_ms:.1f} ms")
            table.set_threads_per_state(0)
        out["bfs"] = bfs

    if not args.no_async:
        # exploration without level barriers vs the level loops, on an
        # uncapped model (same result by definition) and on a chain of
        # one-state levels
        def median_ms(m, t, flags, reps):
            ms, r = [], None
            for i in range(1 + reps):
                r = lhs.reach_explore(m, table=t, flags=flags)
                if i:
                    ms.append(r.gpu_ms)
            return sorted(ms)[len(ms) // 2], r
        reps = max(1, min(args.steps, 3))
        wm = gen.wide_model()
        with lhs.Table(gen.WIDE_TABLE_SLOTS, wm.W) as wt:
            b_ms, rb = median_ms(wm, wt, 0, reps)
            g_ms, rg = median_ms(wm, wt, lhs.REACH_F_GRAPH, reps)
            a_ms, ra = median_ms(wm, wt, lhs.REACH_F_ASYNC, reps)
        nl = {"workload": f"{wm.name}: G(seed={wm.seed}, P={wm.P}, L={wm.L}, S={wm.S}, D={wm.D}, K={wm.K}) "
                          f"explored to exhaustion, table 2^{gen.WIDE_TABLE_SLOTS.bit_length() - 1}",
              "states": ra.total, "edges": ra.edges, "deadlocks": ra.deadlocks, "bfs_levels": rb.n_levels,
              "no_levels_ms": round(a_ms, 2), "states_per_s": round(ra.total / (a_ms / 1e3), 1),
              "level_loop_ms": round(b_ms, 2), "graph_levels_ms": round(g_ms, 2),
              "same_result": (ra.total, ra.edges, ra.deadlocks) == (rb.total, rb.edges, rb.deadlocks) ==
                             (rg.total, rg.edges, rg.deadlocks)}
        golden = os.path.join(ROOT, "tests", "golden", "wide_model.json")
        if os.path.exists(golden):
            with open(golden) as f:
                g = json.load(f)
            nl["matches_oracle"] = (g["total"], g["edges"], g["deadlocks"]) == (ra.total, ra.edges, ra.deadlocks)
        log(f"wide model: level loop {b_ms:.2f} ms, graph levels {g_ms:.2f} ms, no levels {a_ms:.2f} ms")
        if not args.no_chain:
            cm = gen.chain_model()
            with lhs.Table(1 << 16, cm.W) as ct:
                cg_ms, rcg = median_ms(cm, ct, lhs.REACH_F_GRAPH, 1)
                ca_ms, rca = median_ms(cm, ct, lhs.REACH_F_ASYNC, 1)
            nl["chain"] = {"workload": f"chain of {cm.L} one-state levels", "states": rca.total,
                           "no_levels_ms": round(ca_ms, 2), "graph_levels_ms": round(cg_ms, 2),
                           "us_per_state_no_levels": round(ca_ms * 1e3 / rca.total, 2),
                           "same_result": (rca.total, rca.edges) == (rcg.total, rcg.edges)}
            log(f"chain: graph levels {cg_ms:.1f} ms, no levels {ca_ms:.1f} ms")
        out["no_levels"] = nl
    if sweep:
        out["tps_sweep"] = sweep

    table.close()
    del states_d, seen_d, idx_d

    if not args.no_batch:
        models = gen.batch_models()
        batch_cfg, _ = lhs.tune_lookup(lhs.TUNE_BATCH, 32, 1 << 21)
        out["table_shape"]["batch_tables"] = batch_cfg
        tables = [lhs.Table(1 << 21, m.W, lhs.config(**batch_cfg)) for m in models]
        n_states = None

        def run_batch(flags):
            w0 = time.time()
            rs = lhs.reach_explore_batch(models, tables=tables, flags=flags)
            return rs, (time.time() - w0) * 1e3

        def run_alone(flags):
            w0 = time.time()
            rs = [lhs.reach_explore(m, table=t, flags=flags) for m, t in zip(models, tables)]
            return rs, (time.time() - w0) * 1e3

        batch = {}
        for name, fn in (("persistent", lambda: run_batch(0)), ("host_loop", lambda: run_batch(1)),
                         ("one_at_a_time", lambda: run_alone(0)),
                         ("one_at_a_time_graph", lambda: run_alone(lhs.REACH_F_GRAPH))):
            fn()
            times = []
            for _ in range(3):
                rs, wall = fn()
                times.append(wall)
            n_states = sum(r.total for r in rs)
            ms = sorted(times)[1]
            batch[name] = {"wall_ms": round(ms, 2), "states_per_s": round(n_states / (ms / 1e3), 1)}
            if not name.startswith("one_at_a_time"):
                batch[name]["gpu_ms"] = round(rs[0].gpu_ms, 2)
            log(f"batch {name}: {ms:.1f} ms")
        for t in tables:
            t.close()
        batch["workload"] = "64-model mix (gen/manifests/batch_models.json), tables of 2^21 slots"
        batch["states"] = n_states
        best_alone = min(batch["one_at_a_time"]["wall_ms"], batch["one_at_a_time_graph"]["wall_ms"])
        batch["speedup_persistent_vs_one_at_a_time"] = round(best_alone / batch["persistent"]["wall_ms"], 2)
        out["batch"] = batch

    if not args.no_serve:
        models = gen.batch_models()
        n_q = int(args.serve_rate * args.serve_seconds)
        arrivals = gen.poisson_arrivals(0x5E4E, args.serve_rate, n_q)
        picks = (gen.xs64(0x5E4F, n_q) % np.uint64(len(models))).astype(np.int64)
        serve = {"workload": f"Poisson arrivals {args.serve_rate:g}/s for {args.serve_seconds:g} s "
                             f"({n_q} queries) drawn uniformly from the 64-model mix; tables of "
                             f"2^21 slots; latency = result time - scheduled arrival; first "
                             f"{args.serve_warmup:g} s excluded"}
        n_burst = args.serve_burst
        burst_picks = (gen.xs64(0x5E50, n_burst) % np.uint64(len(models))).astype(np.int64) if n_burst else None
        modes = [("continuous", 0, False), ("one_at_a_time", 1, False)]
        if args.serve_rounds:
            modes.append(("continuous_rounds", 0, True))
        for label, max_active, rounds in modes:
            with lhs.Server(capacity=1 << 21, max_active=max_active, rounds=rounds) as srv:
                # resident tables: one warm-up query per shape before the clock starts
                for t in [srv.submit(m) for m in models]:
                    srv.wait(t)
                st0 = srv.stats()
                t0 = srv.clock() + 0.05
                tickets = []
                for i in range(n_q):
                    delay = t0 + arrivals[i] - srv.clock()
                    if delay > 0:
                        time.sleep(delay)
                    tickets.append((i, srv.submit(models[picks[i]])))
                lat, svc, states, done_last = [], [], 0, t0
                for i, t in tickets:
                    r, (sub, adm, done) = srv.wait(t)
                    states += r.total
                    done_last = max(done_last, done)
                    if arrivals[i] >= args.serve_warmup:
                        lat.append((done - (t0 + arrivals[i])) * 1e3)
                        svc.append((done - adm) * 1e3)
                st = srv.stats()
                busy = st["busy_s"] - st0["busy_s"]
                burst = None
                if n_burst:
                    # every query submitted at once: the server, not the
                    # arrival rate, bounds the states per second
                    b0 = srv.clock()
                    bt = [srv.submit(models[k]) for k in burst_picks]
                    b_states, b_last = 0, b0
                    for t in bt:
                        r, (_, _, done) = srv.wait(t)
                        b_states += r.total
                        b_last = max(b_last, done)
                    burst = {"queries": n_burst, "states": int(b_states),
                             "makespan_s": round(b_last - b0, 4),
                             "states_per_s": round(b_states / (b_last - b0), 1)}
            lat, svc = np.array(lat), np.array(svc)
            serve[label] = {"queries": n_q, "states": int(states),
                            "states_per_s": round(states / (done_last - t0), 1),
                            "states_per_busy_s": round(states / busy, 1) if busy > 0 else None,
                            "busy_s": round(busy, 3),
                            "p50_ms": round(float(np.percentile(lat, 50)), 3),
                            "p99_ms": round(float(np.percentile(lat, 99)), 3),
                            "service_p50_ms": round(float(np.percentile(svc, 50)), 3),
                            ("round_steps" if rounds else "launches"): st["steps"] - st0["steps"],
                            "peak_table_bytes": st["peak_bytes"],
                            "burst": burst}
            log(f"serve {label}: p50 {serve[label]['p50_ms']} ms, p99 {serve[label]['p99_ms']} ms, "
                f"busy {busy:.2f} s" + (f", burst {burst['states_per_s']:.3g} states/s" if burst else ""))
        serve["p99_speedup_vs_one_at_a_time"] = round(
            serve["one_at_a_time"]["p99_ms"] / serve["continuous"]["p99_ms"], 2)
        if n_burst:
            serve["burst_speedup_vs_one_at_a_time"] = round(
                serve["continuous"]["burst"]["states_per_s"] / serve["one_at_a_time"]["burst"]["states_per_s"], 2)
        out["serve"] = serve

    if not args.no_cpu:
        import oracle
        S = min(args.cpu_sample, n)
        sample = gen.gather(rows, order[:S])
        c0 = time.time()
        _, _, d = oracle.stream(sample)
        cdt = time.time() - c0
        out["cpu_baseline"] = {"value": round(S / cdt, 1), "unit": "find-or-put ops/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"first {S} rows of the same stream ({d} distinct), "
                                         f"sequential std::unordered_map find-or-put, {cdt:.1f} s"}
        log(f"cpu baseline: {S / cdt:.0f} ops/s over {S} rows")
        if "bfs" in out:
            # the oracle's BFS of the same model to a lower cap (one core)
            mc = gen.big_model(cap=1 << 22)
            c0 = time.time()
            ro = oracle.reach(mc)
            cdt = time.time() - c0
            out["bfs"]["cpu_baseline"] = {
                "value": round(ro.total / cdt, 1), "unit": "states/s", "cores": 1, "kind": "oracle",
                "sample": f"the same model capped at 2^22 states ({ro.total} states, {ro.n_levels} levels, "
                          f"{ro.edges} edges), sequential BFS over std::unordered_set, {cdt:.1f} s"}
            log(f"cpu baseline bfs: {ro.total / cdt:.0f} states/s")
        if "batch" in out:
            # the oracle over the whole 64-model mix, one model after another
            c0 = time.time()
            tot = sum(oracle.reach(m).total for m in gen.batch_models())
            cdt = time.time() - c0
            out["batch"]["cpu_baseline"] = {
                "value": round(tot / cdt, 1), "unit": "states/s", "cores": 1, "kind": "oracle",
                "seconds": round(cdt, 2),
                "sample": f"every model of the 64-model mix ({tot} states), sequential BFS, {cdt:.1f} s"}
            log(f"cpu baseline batch: {cdt:.1f} s for {tot} states")
    if not args.no_cpu_lockless:
        # the paper's method on every host core (multi-core lockless table)
        import cpu_table
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        full = gen.gather(rows, order)
        cpu_table.stream(full[: 1 << 20], args.table_log2 - 8, threads)      # warm-up
        _, _, csec = cpu_table.stream(full, args.table_log2, threads)
        del full
        mb = gen.big_model(cap=1 << 22)
        cr = cpu_table.reach(mb, None, 24, threads)
        out["cpu_lockless"] = {
            "threads": threads,
            "stream_ops_per_s": round(n / csec, 1),
            "stream": f"the same {n}-row stream into a 2^{args.table_log2}-slot table, one pass",
            "bfs_states_per_s": round(cr.total / cr.seconds, 1),
            "bfs": f"the same model capped at 2^22 states ({cr.total} states, {cr.n_levels} levels), "
                   f"table 2^24",
            "gpu_speedup_stream": round(ops_per_s / (n / csec), 2)}
        log(f"cpu lockless ({threads} threads): stream {n / csec:.0f} ops/s, "
            f"bfs {cr.total / cr.seconds:.0f} states/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
