"""The autotuner runs end to end on the GPU (small keys), writes a tuning
file that lhs_tune_load accepts, and its choice is the measured best for
each workload at the chosen line width and probe."""
import json

import pytest

pytestmark = pytest.mark.gpu


def test_autotune_small(tmp_path):
    import torch
    assert torch.cuda.is_available()
    import paper_1004_2772_amd as lhs
    from paper_1004_2772_amd import autotune

    out = tmp_path / "tune.json"
    print("\n[autotune] W=4,16 table 2^14", flush=True)
    doc = autotune.main(["--out", str(out), "--widths", "4,16", "--log2-caps", "14", "--reps", "1",
                         "--no-batch"])
    assert json.loads(out.read_text()) == doc
    assert len(doc["entries"]) == 2
    for e in doc["entries"]:
        assert len(e["stream_ms"]) == len(e["bfs_ms"]) == 36
        ls, probe = e["line_slots"], e["probe"]
        at = {t: e["stream_ms"][f"{ls}/{probe}/{t}"] for t in autotune.TPS}
        bt = {t: e["bfs_ms"][f"{ls}/{probe}/{t}"] for t in autotune.TPS}
        assert at[e["tps_find_or_put"]] == min(at.values())
        assert bt[e["tps_expand"]] == min(bt.values())
        assert e["bfs_model"]["states"] <= e["bfs_model"]["state_cap"]
    try:
        assert lhs.tune_load(str(out)) == 2
        for e in doc["entries"]:
            cfg, found = lhs.tune_lookup(lhs.TUNE_TABLE, e["W"], 1 << 14)
            assert found
            assert cfg == {k: e[k] for k in ("line_slots", "probe", "tps_find_or_put", "tps_expand")}
    finally:
        lhs.tune_clear()
