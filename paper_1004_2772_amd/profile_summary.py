"""Summaries of rocprofv3 result databases (rocpd SQLite) for profiles/.

    python -m paper_1004_2772_amd.profile_summary stats DB [--cmd "..."]
        per-kernel calls / total / average duration (kernel trace)
    python -m paper_1004_2772_amd.profile_summary traffic FETCH_DB WRITE_DB \
        --kernel NAME --ops N --copy-bytes B --sources F1,F2 --out JSON [--cmd "..."]
        FETCH_SIZE / WRITE_SIZE of a kernel per dispatch, scaled by what the
        same counters read for the plain copy probe of B bytes (which reads B
        and writes B bytes), written as JSON for bench.py.
    python -m paper_1004_2772_amd.profile_summary atomics ATOMIC_DB --kernel NAME --ops N \
        --probe NAME --probe-ops M --sources F1,F2 --out JSON [--cmd "..."]
        TCC_ATOMIC_sum (atomic requests at the L2) and TCC_EA0_ATOMIC_sum (atomics
        sent on to memory) of a kernel's largest dispatch and of the random-CAS
        probe's, written as JSON for bench.py (which divides by the launch times).
    python -m paper_1004_2772_amd.profile_summary probes FETCH_DB WRITE_DB --copy-bytes B --out JSON [--cmd "..."]
        FETCH_SIZE / WRITE_SIZE per access of each measurement probe, from the
        timed (second) dispatch of each probe as bench.py runs them: random
        line reads of 64 / 128 / 256 bytes (cooperative lanes), 8-byte slot
        stores, 64-byte row stores, 64-byte row loads and 64-bit CAS; copy-
        calibrated as above.
    python -m paper_1004_2772_amd.profile_summary traffic-sum FETCH_DB WRITE_DB --kernel K1 [--kernel K2] \
        --runs R [--take D1 [--take D2]] --units N --unit-name NAME --copy-bytes B --out JSON [--cmd "..."]
        FETCH_SIZE / WRITE_SIZE summed over the dispatches of the named kernels
        (of each, the first D in dispatch order: one --take per kernel, or one
        for all; default all), divided by R (the program ran the same work R
        times in them), scaled by the copy probe as above; per run and per
        unit (e.g. per edge of an exploration).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "")
    return n.split("(")[0] if "(" in n else n


def kernel_stats(db: str):
    """Per kernel: calls, total/avg/min/max duration, and the average over the
    dispatches with the kernel's largest grid (separates e.g. the 2^26-row
    find-or-put launches from one-row inserts of the same kernel)."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(duration), avg(duration), min(duration), "
                       "max(duration), max(grid_x) from kernels group by name "
                       "order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1
    out = []
    for r in rows:
        big = con.execute("select count(*), avg(duration) from kernels where name = ? and grid_x = ?",
                          (r[0], r[6])).fetchone()
        out.append(dict(kernel=_short(r[0]), calls=r[1], total_ms=r[2] / 1e6, avg_ms=r[3] / 1e6,
                        min_ms=r[4] / 1e6, max_ms=r[5] / 1e6, pct=100.0 * r[2] / total,
                        big_grid=r[6], big_calls=big[0], big_avg_ms=big[1] / 1e6))
    return out


def counter_per_dispatch(db: str, counter: str):
    """{short kernel name: [(grid size, value) per dispatch, ...]}"""
    con = sqlite3.connect(db)
    out = {}
    for name, grid, val in con.execute("select kernel_name, grid_size, value from counters_collection "
                                       "where counter_name = ? order by dispatch_id", (counter,)):
        out.setdefault(_short(name), []).append((grid, val))
    return out


def largest_dispatch(rows):
    """Counter value of the dispatch with the largest grid (the last such)."""
    g = max(r[0] for r in rows)
    return [r[1] for r in rows if r[0] == g][-1]


def sources_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--cmd", default="")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_db")
    t.add_argument("write_db")
    t.add_argument("--kernel", required=True)
    t.add_argument("--ops", type=int, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--sources", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--cmd", default="")
    t.add_argument("--summary", default="")
    at = sub.add_parser("atomics")
    at.add_argument("db")
    at.add_argument("--kernel", required=True)
    at.add_argument("--ops", type=int, required=True)
    at.add_argument("--probe", required=True)
    at.add_argument("--probe-ops", type=int, required=True)
    at.add_argument("--sources", required=True)
    at.add_argument("--out", required=True)
    at.add_argument("--cmd", default="")
    pr = sub.add_parser("probes")
    pr.add_argument("fetch_db")
    pr.add_argument("write_db")
    pr.add_argument("--copy-bytes", type=int, required=True)
    pr.add_argument("--out", required=True)
    pr.add_argument("--cmd", default="")
    ts = sub.add_parser("traffic-sum")
    ts.add_argument("fetch_db")
    ts.add_argument("write_db")
    ts.add_argument("--kernel", action="append", required=True)
    ts.add_argument("--runs", type=int, required=True)
    ts.add_argument("--take", type=int, action="append", default=[])
    ts.add_argument("--units", type=int, required=True)
    ts.add_argument("--unit-name", default="units")
    ts.add_argument("--copy-bytes", type=int, required=True)
    ts.add_argument("--out", required=True)
    ts.add_argument("--cmd", default="")
    a = ap.parse_args(argv)

    if a.mode == "stats":
        if a.cmd:
            print(f"# command: {a.cmd}")
        print(f"{'kernel':44s} {'calls':>6s} {'total_ms':>10s} {'avg_ms':>9s} {'min_ms':>9s} "
              f"{'max_ms':>9s} {'%':>6s}  {'largest-grid calls':>18s} {'avg_ms':>9s}")
        for r in kernel_stats(a.db):
            print(f"{r['kernel'][:44]:44s} {r['calls']:6d} {r['total_ms']:10.3f} {r['avg_ms']:9.4f} "
                  f"{r['min_ms']:9.4f} {r['max_ms']:9.4f} {r['pct']:6.2f}  {r['big_calls']:18d} "
                  f"{r['big_avg_ms']:9.4f}")
        return

    if a.mode == "atomics":
        res = dict(kernel=a.kernel, ops_per_launch=a.ops, probe=a.probe, probe_ops_per_launch=a.probe_ops,
                   source_sha=sources_sha(a.sources.split(",")), command=a.cmd)
        for counter, key in (("TCC_ATOMIC_sum", "l2_atomics"), ("TCC_EA0_ATOMIC_sum", "ea_atomics")):
            per = counter_per_dispatch(a.db, counter)
            if a.kernel not in per or a.probe not in per:
                sys.exit(f"{counter}: kernel or probe missing from {a.db}")
            res[f"{key}_per_launch"] = largest_dispatch(per[a.kernel])
            res[f"probe_{key}_per_launch"] = largest_dispatch(per[a.probe])
            res[f"{key}_per_op"] = res[f"{key}_per_launch"] / a.ops
            res[f"probe_{key}_per_op"] = res[f"probe_{key}_per_launch"] / a.probe_ops
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res, indent=1))
        return

    fetch = counter_per_dispatch(a.fetch_db, "FETCH_SIZE")
    write = counter_per_dispatch(a.write_db, "WRITE_SIZE")
    if a.mode == "probes":
        if not fetch.get("k_probe_copy") or not write.get("k_probe_copy"):
            sys.exit("copy probe missing from the counter runs (run bench.py with --calib-copy)")
        f_fetch = a.copy_bytes / (largest_dispatch(fetch["k_probe_copy"]) * 1024.0)
        f_write = a.copy_bytes / (largest_dispatch(write["k_probe_copy"]) * 1024.0)
        # bench.py's probe order: each probe runs twice (warm-up, timed)
        plan = [("random_64B_line_read", "void k_probe_lines_coop<4u>", 1, 1 << 25),
                ("random_128B_line_read", "void k_probe_lines_coop<8u>", 1, 1 << 24),
                ("random_256B_line_read", "void k_probe_lines_coop<16u>", 1, 1 << 23),
                ("slot_store_8B", "void k_probe_access<0u>", 1, 1 << 27),
                ("row_store_64B", "void k_probe_access<1u>", 1, 1 << 27),
                ("row_load_64B", "void k_probe_access<2u>", 1, 1 << 27),
                ("cas_64bit", "k_probe_cas", 1, 1 << 26)]
        res = dict(fetch_scale=f_fetch, write_scale=f_write, command=a.cmd, per_access={})
        for name, kernel, k, ops in plan:
            fl, wl = fetch.get(kernel, []), write.get(kernel, [])
            if len(fl) <= k or len(wl) <= k:
                sys.exit(f"{kernel}: dispatch {k} missing from the counter runs")
            res["per_access"][name] = {
                "accesses": ops,
                "fetch_bytes": fl[k][1] * 1024.0 * f_fetch / ops,
                "write_bytes": wl[k][1] * 1024.0 * f_write / ops}
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res, indent=1))
        return
    if a.mode == "traffic-sum":
        if not fetch.get("k_probe_copy") or not write.get("k_probe_copy"):
            sys.exit("copy probe missing from the counter runs (run bench.py with --calib-copy)")
        f_fetch = a.copy_bytes / (largest_dispatch(fetch["k_probe_copy"]) * 1024.0)
        f_write = a.copy_bytes / (largest_dispatch(write["k_probe_copy"]) * 1024.0)
        names = a.kernel
        missing = [n for n in names if n not in fetch or n not in write]
        if missing:
            sys.exit(f"kernels missing from the counter runs: {missing}")
        takes = a.take or [0]
        if len(takes) == 1:
            takes = takes * len(names)
        if len(takes) != len(names):
            sys.exit("give one --take per --kernel, or one for all")
        fl = [v for n, k in zip(names, takes) for _, v in fetch[n][:k or None]]
        wl = [v for n, k in zip(names, takes) for _, v in write[n][:k or None]]
        kf, kw = sum(fl) / a.runs, sum(wl) / a.runs
        res = dict(kernels=names, takes=takes, runs=a.runs, dispatches_per_run=len(fl) / a.runs,
                   fetch_scale=f_fetch, write_scale=f_write,
                   fetch_bytes_per_run=kf * 1024.0 * f_fetch, write_bytes_per_run=kw * 1024.0 * f_write,
                   units_per_run=a.units, unit=a.unit_name, command=a.cmd)
        res[f"fetch_bytes_per_{a.unit_name}"] = res["fetch_bytes_per_run"] / a.units
        res[f"write_bytes_per_{a.unit_name}"] = res["write_bytes_per_run"] / a.units
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res, indent=1))
        return
    copy_f = fetch.get("k_probe_copy")
    copy_w = write.get("k_probe_copy")
    if not copy_f or not copy_w:
        sys.exit("copy probe missing from the counter runs (run bench.py with --calib-copy)")
    cf, cw = largest_dispatch(copy_f), largest_dispatch(copy_w)
    f_fetch = a.copy_bytes / (cf * 1024.0)
    f_write = a.copy_bytes / (cw * 1024.0)
    kf = largest_dispatch(fetch[a.kernel])
    kw = largest_dispatch(write[a.kernel])
    res = dict(kernel=a.kernel, ops_per_launch=a.ops, fetch_kib=kf, write_kib=kw,
               copy_bytes=a.copy_bytes, copy_fetch_kib=cf, copy_write_kib=cw,
               fetch_scale=f_fetch, write_scale=f_write,
               fetch_bytes=kf * 1024.0 * f_fetch, write_bytes=kw * 1024.0 * f_write,
               source_sha=sources_sha(a.sources.split(",")), command=a.cmd, summary=a.summary)
    res["fetch_bytes_per_op"] = res["fetch_bytes"] / a.ops
    res["write_bytes_per_op"] = res["write_bytes"] / a.ops
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
