"""Select the seeds of the large model and of the 64-model batch mix.

Inputs only (no expected values are stored here).  Uses the generators in gen/
and measures candidate state-space sizes with the CPU oracle:

* big_model.json  — G(seed, P=12, L=16, S=4, D=10, K=3): the first seed in
  1, 2, 3, ... whose reachable set exceeds the 2^20-state probe cap (the
  generator is bimodal: a model either dies within a few hundred states or
  keeps growing; the full 2^27-cap run is recorded by tests/golden/make_golden.py,
  which also confirms that the 2^27 cap fires).
* batch_models.json — candidates drawn by gen.draw_batch_params(0xC4C4C4C4, t)
  for t = 0, 1, 2, ...; a candidate is accepted when its full reachable set has
  between 10^3 and 10^6 states; acceptance is stratified by decade (21 models
  in [10^3, 10^4), 21 in [10^4, 10^5), 22 in [10^5, 10^6]) so the mix spans the
  whole size range, taking the earliest accepted trials of each decade.

Run:  python gen/manifests/make_manifests.py   (about 3 minutes on 8 cores)
"""
import json
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen      # noqa: E402
import oracle   # noqa: E402

MASTER = 0xC4C4C4C4
QUOTA = {4: 21, 5: 21, 6: 22}     # decimal digits of |R| -> count


def _probe(trial):
    p = gen.draw_batch_params(MASTER, trial)
    m = gen.guarded_model(p["seed"], p["P"], p["L"], p["S"], p["D"], p["K"])
    r = oracle.reach(m, cap=10 ** 6 + 1)
    return trial, p, r.total, r.capped


def big_model():
    D = 10
    for seed in range(1, 1000):
        m = gen.guarded_model(seed, gen.BIG_P, gen.BIG_L, gen.BIG_S, D, gen.BIG_K)
        if oracle.reach(m, cap=1 << 20).capped:
            return dict(seed=hex(seed), D=D, P=gen.BIG_P, L=gen.BIG_L, S=gen.BIG_S, K=gen.BIG_K,
                        rule="first seed from 1 whose reachable set exceeds 2^20 states")
    raise RuntimeError("no exploding seed found")


def batch_models():
    got = {k: [] for k in QUOTA}
    trial = 0
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        while any(len(got[k]) < QUOTA[k] for k in QUOTA):
            for t, p, total, capped in pool.map(_probe, range(trial, trial + 512), chunksize=8):
                d = len(str(total))
                if not capped and 10 ** 3 <= total <= 10 ** 6 and d in got and len(got[d]) < QUOTA[d]:
                    got[d].append(dict(trial=t, name=f"mix{t}", seed=hex(p["seed"]), P=p["P"],
                                       L=p["L"], S=p["S"], D=p["D"], K=p["K"], states=total))
            trial += 512
    models = sorted((m for v in got.values() for m in v), key=lambda m: m["trial"])
    return dict(master_seed=hex(MASTER), trials_scanned=trial, quota=QUOTA, models=models)


if __name__ == "__main__":
    big = big_model()
    with open(os.path.join(HERE, "big_model.json"), "w") as f:
        json.dump(big, f, indent=1)
    print("big model", big, flush=True)
    mix = batch_models()
    with open(os.path.join(HERE, "batch_models.json"), "w") as f:
        json.dump(mix, f, indent=1)
    print("batch models:", len(mix["models"]), "states", sum(m["states"] for m in mix["models"]))
