"""Write the expected results of the large workloads, computed by the CPU
oracle only (no GPU code is imported).

* big_model.json   — the 12-process x 16-local model of gen/manifests, BFS
                     capped at 2^27 states (level-prefix cap): per-level
                     counts, edges, deadlocks, and the oracle's set digest.
* batch_models.json — full (uncapped) results of each of the 64 models of the
                     batch mix.
* wide_model.json  — the uncapped 8-process x 6-local model (gen.wide_model),
                     explored to exhaustion: per-level counts, edges,
                     deadlocks and the set digest.

Run:  python tests/golden/make_golden.py [big|batch|wide|all]
(the 2^27 run needs about 16 GB of host memory and a few minutes).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import gen      # noqa: E402
import oracle   # noqa: E402


def _entry(m, r, secs):
    return dict(name=m.name, seed=hex(m.seed), P=m.P, L=m.L, S=m.S, D=m.D, K=m.K, W=m.W,
                cap=m.cap, total=r.total, n_levels=r.n_levels, level_counts=r.level_counts,
                edges=r.edges, deadlocks=r.deadlocks, capped=r.capped,
                digest=[r.digest[0], hex(r.digest[1]), hex(r.digest[2])], oracle_seconds=round(secs, 2))


def big():
    m = gen.big_model()
    t = time.time()
    r = oracle.reach(m)
    e = _entry(m, r, time.time() - t)
    with open(os.path.join(HERE, "big_model.json"), "w") as f:
        json.dump(e, f, indent=1)
    print("big", e["total"], e["n_levels"], e["edges"], e["capped"], e["oracle_seconds"], flush=True)


def batch():
    out = []
    for m in gen.batch_models():
        t = time.time()
        r = oracle.reach(m)
        out.append(_entry(m, r, time.time() - t))
    with open(os.path.join(HERE, "batch_models.json"), "w") as f:
        json.dump(dict(models=out), f, indent=1)
    print("batch", len(out), sum(e["total"] for e in out), flush=True)


def wide():
    m = gen.wide_model()
    t = time.time()
    r = oracle.reach(m)
    e = _entry(m, r, time.time() - t)
    with open(os.path.join(HERE, "wide_model.json"), "w") as f:
        json.dump(e, f, indent=1)
    print("wide", e["total"], e["n_levels"], e["edges"], e["capped"], e["oracle_seconds"], flush=True)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("wide", "all"):
        wide()
    if what in ("batch", "all"):
        batch()
    if what in ("big", "all"):
        big()
