"""Speedup and efficiency over workers: the paper's scalability measurement
(speedup S = T_1 / T_N and efficiency E = S / N over N workers, section
"Preliminaries"; write-busy waits per run, the figure on lock hits) taken on
one GPU and on the host's cores.

    python -m paper_1004_2772_amd.scaling [--out JSON] [--txt TABLE] [--quick]

GPU: a worker is a workgroup of 256 lanes that expands states
(lhs_set_workers caps how many a launch uses); N = 1 .. every workgroup that
fits on the GPU at once (1024 on MI355X).  Workloads: the 12x16 model's level-synchronous BFS
capped at 2^22 states and the 1.08M-state G(77,7,6,3,4,2) model explored
without levels.  The batched find-or-put has no worker count of its own (one
workgroup per 256 operations) and is not part of this measurement.

CPU: the multi-core lockless table (cpu_table) with N = 1 .. nproc threads on
a find-or-put stream and the same BFS capped at 2^20 states.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from . import REACH_F_ASYNC, Table, reach_explore, tune_load_default

STREAM_W = 16
BFS_CAP = 1 << 22


def log(msg):
    print(f"[scaling {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def gpu_points(workers: list[int], reps: int) -> list[dict]:
    import gen
    big = gen.big_model(cap=BFS_CAP)
    mid = gen.guarded_model(77, 7, 6, 3, 4, 2)
    out = []
    med = lambda xs: sorted(xs[1:])[len(xs[1:]) // 2]
    with Table(1 << 24, big.W) as tb, Table(1 << 22, mid.W) as tm:
        for n in workers:
            tb.set_workers(n)
            tm.set_workers(n)
            bfs, nol = [], []
            for _ in range(reps + 1):
                r = reach_explore(big, table=tb)
                bfs.append(r.gpu_ms)
            for _ in range(reps + 1):
                a = reach_explore(mid, cap=0, table=tm, flags=REACH_F_ASYNC)
                nol.append(a.gpu_ms)
            p = {"workers": n, "bfs_ms": round(med(bfs), 3), "bfs_Mstates_per_s": round(r.total / med(bfs) / 1e3, 2),
                 "bfs_states": r.total, "bfs_levels": r.level_counts, "bfs_wait_hits": r.wait_hits,
                 "no_levels_ms": round(med(nol), 3), "no_levels_Mstates_per_s": round(a.total / med(nol) / 1e3, 2),
                 "no_levels_states": a.total, "no_levels_edges": a.edges, "no_levels_wait_hits": a.wait_hits}
            out.append(p)
            log(f"{n} workgroups: BFS {p['bfs_Mstates_per_s']} M states/s, "
                f"no levels {p['no_levels_Mstates_per_s']} M states/s")
        tb.set_workers(0)
        tm.set_workers(0)
    base = out[0]
    for p in out:
        k = p["workers"] / base["workers"]
        for key, tkey in (("bfs", "bfs_ms"), ("no_levels", "no_levels_ms")):
            s = base[tkey] / p[tkey]
            p[f"{key}_speedup"] = round(s, 3)
            p[f"{key}_efficiency"] = round(s / k, 3)
    return out


def cpu_points(threads: list[int]) -> list[dict]:
    import cpu_table
    import gen
    rows, order = gen.dup_stream(0x5CA1AB1E, 1 << 21, STREAM_W, 2)
    full = gen.gather(rows, order)
    big = gen.big_model(cap=1 << 20)
    out = []
    for t in threads:
        _, _, ssec = cpu_table.stream(full, 23, t)
        r = cpu_table.reach(big, None, 22, t)
        out.append({"threads": t, "stream_s": round(ssec, 4), "stream_Mops": round(len(full) / ssec / 1e6, 2),
                    "bfs_s": round(r.seconds, 4), "bfs_Mstates_per_s": round(r.total / r.seconds / 1e6, 2)})
        log(f"{t} threads: stream {out[-1]['stream_Mops']} M ops/s, BFS {out[-1]['bfs_Mstates_per_s']} M states/s")
    for p in out:
        for key, tkey in (("stream", "stream_s"), ("bfs", "bfs_s")):
            s = out[0][tkey] / p[tkey]
            p[f"{key}_speedup"] = round(s, 3)
            p[f"{key}_efficiency"] = round(s / (p["threads"] / out[0]["threads"]), 3)
    return out


def tables_text(res: dict, command: str) -> str:
    lines = ["# speedup S = T_1 / T_N and efficiency E = S / N over N workers (MI355X, one GPU; host cores)",
             f"# command: {command}",
             "# GPU: N workgroups of 256 lanes expanding states (lhs_set_workers); CPU: N threads of the",
             "# multi-core lockless table; waits = write-busy hits of the run", ""]
    lines.append("GPU workgroups  BFS M states/s      S       E    waits | no levels M states/s      S       E    waits")
    for p in res["gpu"]:
        lines.append(f"     {p['workers']:9d}  {p['bfs_Mstates_per_s']:13.2f}  {p['bfs_speedup']:7.2f} "
                     f"{p['bfs_efficiency']:6.3f} {p['bfs_wait_hits']:8d} | {p['no_levels_Mstates_per_s']:19.2f}  "
                     f"{p['no_levels_speedup']:7.2f} {p['no_levels_efficiency']:6.3f} {p['no_levels_wait_hits']:8d}")
    lines.append("")
    lines.append("CPU threads  stream M ops/s   S     E  |  BFS M states/s   S     E")
    for p in res["cpu"]:
        lines.append(f"     {p['threads']:4d}  {p['stream_Mops']:12.2f}  {p['stream_speedup']:6.2f} "
                     f"{p['stream_efficiency']:5.2f} |  {p['bfs_Mstates_per_s']:12.2f}  {p['bfs_speedup']:6.2f} "
                     f"{p['bfs_efficiency']:5.2f}")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="")
    ap.add_argument("--txt", default="")
    ap.add_argument("--quick", action="store_true", help="two worker counts, two thread counts, one rep")
    ap.add_argument("--no-cpu", action="store_true")
    a = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the scaling runs time kernels on a GPU")
    tune_load_default()
    # 1024 = 4 workgroups on each of 256 compute units, what fits at once
    workers = [4, 256] if a.quick else [1, 4, 16, 64, 256, 1024]
    nproc = min(os.cpu_count() or 1, 16)
    threads = [1, nproc] if a.quick else sorted({1, 2, 4, 8, nproc})
    t0 = time.time()
    res = {"gpu": gpu_points(workers, 1 if a.quick else 3)}
    res["cpu"] = [] if a.no_cpu else cpu_points(threads)
    res["seconds"] = round(time.time() - t0, 1)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    if a.txt:
        if not res["cpu"]:
            res["cpu"] = []
        with open(a.txt, "w") as f:
            f.write(tables_text(res, " ".join(["python -m paper_1004_2772_amd.scaling"] + (argv or sys.argv[1:]))))
    return res


if __name__ == "__main__":
    main()
