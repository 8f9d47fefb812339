"""Find-or-put throughput against fill rate, table size, read/write ratio and
vector size: the paper's synthetic table experiment (section "Shared
Storage Parameters", figure "Effect of fill-rate and size/rw-write on
average throughput"), on one GPU.

    python -m paper_1004_2772_amd.sweep [--out JSON] [--txt TABLE] [--quick]

For each (W, table size 2^c, reads per write n) a table is filled band by
band up to 99.9 % of its slots.  A band inserts its share of seeded distinct
vectors and, mixed in at random positions, looks up n times as many vectors
drawn uniformly from those stored before the band (capped at 2^24 reads per
band); each band is one find-or-put call, timed with HIP events, into a
table of the tuned shape.  A second, identical fill of a fresh table counts
the lines each band's operations probe (and the waits and CAS retries): the
count is one atomic per wavefront on one address, which would slow the timed
pass.  Every band of both passes is checked: inserted rows must report new,
looked-up rows seen, and the table count must equal the rows inserted so far.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import Table, tune_load_default

BANDS = [0.5, 0.75, 0.9, 0.95, 0.99, 0.999]
MAX_READS = 1 << 24


def log(msg):
    print(f"[sweep {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def run_one(W: int, log2cap: int, n_reads: int, seed: int, count_lines: bool = False) -> list:
    import torch

    import gen
    cap = 1 << log2cap
    total = int(cap * BANDS[-1])
    rows, _ = gen.dup_stream(seed, total, W, 1)        # distinct rows, insertion order
    out = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with Table(cap, W) as t:
        if count_lines:
            t.set_counters(1)      # lines probed per operation
        lines_before = waits_before = cas_before = 0
        lo = 0
        for b, frac in enumerate(BANDS):
            hi = int(cap * frac)
            nw = hi - lo
            nr = min(n_reads * nw, MAX_READS) if lo > 0 else 0
            # positions of the reads among the band's operations, and which
            # stored rows they look up (seeded, from the generator module)
            read_rows = (gen.xs64(seed * 31 + b, nr) % np.uint64(lo)).astype(np.int64) if nr else None
            ops = nw + nr
            perm = gen.permutation(seed * 17 + b, ops).astype(np.int64)
            src = np.empty(ops, dtype=np.int64)
            src[perm[:nw]] = np.arange(lo, hi)
            is_write = np.zeros(ops, dtype=bool)
            is_write[perm[:nw]] = True
            if nr:
                src[perm[nw:]] = read_rows
            batch = torch.from_numpy(gen.gather(rows, src.astype(np.uint32)).view(np.int32)).cuda()
            seen = torch.empty(ops, dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
            e0.record()
            t.find_or_put(batch, seen)
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            t.check()
            seen_h = seen.cpu().numpy()
            ok = bool(np.all(seen_h[is_write] == 0) and np.all(seen_h[~is_write] == 1))
            stored = t.count()
            ok = ok and stored == hi
            info = t.info()
            lines, waits, cas = info["lines_probed"], info["wait_hits"], info["cas_failures"]
            band = {"fill_from": round(lo / cap, 4), "fill_to": frac, "writes": nw, "reads": nr,
                    "ms": round(ms, 4), "Gops": round(ops / ms / 1e6, 3),
                    "wait_hits": waits - waits_before, "cas_failures": cas - cas_before, "ok": ok}
            if count_lines:
                band["lines_per_op"] = round((lines - lines_before) / ops, 3)
            out.append(band)
            lines_before, waits_before, cas_before = lines, waits, cas
            if not ok:
                raise RuntimeError(f"sweep W={W} 2^{log2cap} n={n_reads} band {frac}: wrong seen flags "
                                   f"or count {stored} != {hi}")
            lo = hi
            del batch, seen
    torch.cuda.empty_cache()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="")
    ap.add_argument("--quick", action="store_true", help="small sizes only")
    ap.add_argument("--txt", default="", help="also write the G ops/s and lines-per-op tables")
    a = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the sweep times kernels on a GPU")
    tune_load_default()     # tables take the tuned shapes, as the benchmark's do
    if a.quick:
        points = [(W, c, n) for W in (4, 16) for c in (16,) for n in (0, 2)]
    else:
        points = [(W, c, n) for W in (4, 16, 32) for c in (20, 24, 27) for n in (0, 1, 4)
                  if not (W == 32 and c == 27)]
    res = {"bands": BANDS, "max_reads_per_band": MAX_READS, "points": []}
    t0 = time.time()
    for i, (W, c, n) in enumerate(points):
        bands = run_one(W, c, n, 1000 + i)
        counted = run_one(W, c, n, 1000 + i, count_lines=True)
        for b, cb in zip(bands, counted):
            b["lines_per_op"] = cb["lines_per_op"]
        res["points"].append({"W": W, "log2_capacity": c, "reads_per_write": n, "bands": bands})
        log(f"W={W} 2^{c} n={n}: " + " ".join(f"{b['fill_to']:.3f}:{b['Gops']:.2f}" for b in bands))
    res["seconds"] = round(time.time() - t0, 1)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    if a.txt:
        with open(a.txt, "w") as f:
            f.write(tables_text(res, " ".join(["python -m paper_1004_2772_amd.sweep"] + (argv or sys.argv[1:]))))
    return res


def tables_text(res: dict, command: str) -> str:
    """Throughput (G ops/s) and lines probed per operation by fill band."""
    head = "".join(f"{b:>8}" for b in res["bands"])
    out = [f"# find-or-put by fill band: table of the tuned shape, one call per band (MI355X, one GPU)",
           f"# command: {command}",
           f"# bands end at fill {res['bands']}; reads per band capped at {res['max_reads_per_band']}; "
           f"every band checked (new/seen flags, count); {res['seconds']} s",
           "# lines per op from a second, identical fill with the line counter on", ""]
    for key, title, fmt in (("Gops", "G ops/s", "{:8.2f}"), ("lines_per_op", "lines probed per operation", "{:8.2f}")):
        out.append(f"{title}:")
        out.append(f"  W log2cap reads/write{head}")
        for p in res["points"]:
            out.append(f"{p['W']:>3} {p['log2_capacity']:>6} {p['reads_per_write']:>11}" +
                       "".join(fmt.format(b[key]) for b in p["bands"]))
        out.append("")
    return "\n".join(out)


if __name__ == "__main__":
    main()
