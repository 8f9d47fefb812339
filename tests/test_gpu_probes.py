"""The measurement probes touch what they claim: the store forms write their
rows and slots at random positions of the buffer, the load forms leave it
unchanged."""
import pytest

pytestmark = pytest.mark.gpu

import paper_1004_2772_amd as lhs


def test_random_access_forms():
    import torch
    assert torch.cuda.is_available()
    dev = torch.device("cuda", 0)
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    rows, ops = 1 << 14, 1000
    print(f"\n[probes] random access forms: {rows} rows, {ops} ops", flush=True)
    buf = torch.zeros(rows * 8, dtype=torch.int64, device=dev)
    lhs.probe_random_access(buf, "row_store", ops, 7, sink)
    torch.cuda.synchronize()
    r = buf.view(rows, 8).cpu()
    written = (r != 0).any(dim=1)
    # every row is untouched or holds its op's value in all eight words
    assert bool(((r == r[:, :1]).all(dim=1) | ~written).all())
    n = int(written.sum())
    assert 900 <= n <= ops          # ~970 distinct rows expected from 1000 random draws
    before = buf.clone()
    lhs.probe_random_access(buf, "row_load", ops, 7, sink)
    torch.cuda.synchronize()
    assert torch.equal(buf, before)
    buf.zero_()
    lhs.probe_random_access(buf, "slot_store", ops, 9, sink)
    torch.cuda.synchronize()
    s = buf.cpu()
    nz = s[s != 0]
    assert 950 <= nz.numel() <= ops and bool((nz & 1 == 1).all())    # r | 1 at random slots
    lhs.probe_random_lines(buf, 64, 4, ops, 1, sink)
    lhs.probe_random_cas(buf, ops, 3, sink)
    torch.cuda.synchronize()
