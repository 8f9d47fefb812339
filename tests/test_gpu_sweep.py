"""The fill-rate / size / read-write / vector-size sweep runs on the GPU and
checks every band (inserted rows new, looked-up rows seen, counts), up to
99.9 % fill."""
import pytest

pytestmark = pytest.mark.gpu


def test_sweep_quick():
    import torch
    assert torch.cuda.is_available()
    from paper_1004_2772_amd import sweep
    print("\n[sweep] quick", flush=True)
    res = sweep.main(["--quick"])
    assert len(res["points"]) == 4
    for p in res["points"]:
        assert [b["fill_to"] for b in p["bands"]] == sweep.BANDS
        assert all(b["ok"] for b in p["bands"])
        assert p["bands"][-1]["writes"] > 0
        lines = [b["lines_per_op"] for b in p["bands"]]
        # probe lengths grow with the fill: about one line per operation
        # while the table is at most half full, many near 99.9 %
        assert 1.0 <= lines[0] <= 1.1
        assert all(a <= b * 1.05 for a, b in zip(lines, lines[1:]))
        assert lines[-1] > 5 * lines[0]
