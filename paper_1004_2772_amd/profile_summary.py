"""Summaries of rocprofv3 result databases (rocpd SQLite) for profiles/.

    python -m paper_1004_2772_amd.profile_summary stats DB [--cmd "..."]
        per-kernel calls / total / average duration (kernel trace)
    python -m paper_1004_2772_amd.profile_summary traffic FETCH_DB WRITE_DB \
        --kernel NAME --ops N --copy-bytes B --sources F1,F2 --out JSON [--cmd "..."]
        FETCH_SIZE / WRITE_SIZE of a kernel per dispatch, scaled by what the
        same counters read for the plain copy probe of B bytes (which reads B
        and writes B bytes), written as JSON for bench.py.
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
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(duration), avg(duration), min(duration), "
                       "max(duration) from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1
    return [dict(kernel=_short(r[0]), calls=r[1], total_ms=r[2] / 1e6, avg_ms=r[3] / 1e6,
                 min_ms=r[4] / 1e6, max_ms=r[5] / 1e6, pct=100.0 * r[2] / total) for r in rows]


def counter_per_dispatch(db: str, counter: str):
    """{short kernel name: [value per dispatch, ...]}"""
    con = sqlite3.connect(db)
    out = {}
    for name, val in con.execute("select kernel_name, value from counters_collection "
                                 "where counter_name = ? order by dispatch_id", (counter,)):
        out.setdefault(_short(name), []).append(val)
    return out


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
    a = ap.parse_args(argv)

    if a.mode == "stats":
        if a.cmd:
            print(f"# command: {a.cmd}")
        print(f"{'kernel':60s} {'calls':>6s} {'total_ms':>10s} {'avg_ms':>9s} {'min_ms':>9s} {'max_ms':>9s} {'%':>6s}")
        for r in kernel_stats(a.db):
            print(f"{r['kernel'][:60]:60s} {r['calls']:6d} {r['total_ms']:10.3f} {r['avg_ms']:9.4f} "
                  f"{r['min_ms']:9.4f} {r['max_ms']:9.4f} {r['pct']:6.2f}")
        return

    fetch = counter_per_dispatch(a.fetch_db, "FETCH_SIZE")
    write = counter_per_dispatch(a.write_db, "WRITE_SIZE")
    copy_f = fetch.get("k_probe_copy")
    copy_w = write.get("k_probe_copy")
    if not copy_f or not copy_w:
        sys.exit("copy probe missing from the counter runs (run bench.py with --calib-copy)")
    f_fetch = a.copy_bytes / (copy_f[-1] * 1024.0)
    f_write = a.copy_bytes / (copy_w[-1] * 1024.0)
    kf = fetch[a.kernel][-1]
    kw = write[a.kernel][-1]
    res = dict(kernel=a.kernel, ops_per_launch=a.ops, fetch_kib=kf, write_kib=kw,
               copy_bytes=a.copy_bytes, copy_fetch_kib=copy_f[-1], copy_write_kib=copy_w[-1],
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
