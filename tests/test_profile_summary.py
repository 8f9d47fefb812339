"""The arithmetic of the counter summaries behind the committed traffic
figures, on small synthetic databases with the counter table layout of
rocprofv3 (no GPU)."""
import json
import sqlite3

from paper_1004_2772_amd import profile_summary as ps

K = "void (anonymous namespace)::k_work<1, 8u>(int*)"
COPY = "(anonymous namespace)::k_probe_copy(uint4*, uint4 const*, unsigned long)"


def _db(path, counter, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, grid_size integer, "
                "counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?, ?)",
                    [(i, n, g, counter, v) for i, (n, g, v) in enumerate(rows)])
    con.commit()
    con.close()
    return str(path)


def test_traffic_scales_by_the_copy_probe(tmp_path):
    copy_bytes = 1 << 20
    # the copy reads and writes copy_bytes; its counters read half and all of it
    f = _db(tmp_path / "f.db", "FETCH_SIZE", [(COPY, 4096, copy_bytes / 2048), (K, 256, 10.0), (K, 65536, 300.0)])
    w = _db(tmp_path / "w.db", "WRITE_SIZE", [(COPY, 4096, copy_bytes / 1024), (K, 256, 1.0), (K, 65536, 100.0)])
    out = tmp_path / "t.json"
    ps.main(["traffic", f, w, "--kernel", "void k_work<1, 8u>", "--ops", "1000", "--copy-bytes", str(copy_bytes),
             "--sources", "bench.py", "--out", str(out)])
    r = json.loads(out.read_text())
    assert r["fetch_scale"] == 2.0 and r["write_scale"] == 1.0
    # the largest-grid dispatch is the one summarised
    assert r["fetch_bytes"] == 300 * 1024 * 2.0 and r["write_bytes"] == 100 * 1024
    assert r["fetch_bytes_per_op"] == 614.4 and r["write_bytes_per_op"] == 102.4


def test_traffic_sum_takes_the_first_dispatches_of_the_runs(tmp_path):
    copy_bytes = 1 << 20
    runs = [(K, 1024, v) for v in (1.0, 2.0, 3.0)] * 2 + [(K, 1024, 1000.0)]   # two runs, then other work
    f = _db(tmp_path / "f.db", "FETCH_SIZE", [(COPY, 4096, copy_bytes / 2048)] + runs)
    w = _db(tmp_path / "w.db", "WRITE_SIZE", [(COPY, 4096, copy_bytes / 1024)] + runs)
    out = tmp_path / "s.json"
    ps.main(["traffic-sum", f, w, "--kernel", "void k_work<1, 8u>", "--runs", "2", "--take", "6",
             "--units", "3", "--unit-name", "edge", "--copy-bytes", str(copy_bytes), "--out", str(out)])
    r = json.loads(out.read_text())
    assert r["dispatches_per_run"] == 3
    assert r["fetch_bytes_per_run"] == 6 * 1024 * 2.0 and r["write_bytes_per_run"] == 6 * 1024
    assert r["fetch_bytes_per_edge"] == 4096 and r["write_bytes_per_edge"] == 2048


def test_probes_take_the_timed_dispatch_of_each_probe(tmp_path):
    copy_bytes = 1 << 20
    lines = {4: 1 << 25, 8: 1 << 24, 16: 1 << 23}
    rows = [(COPY, 4096, copy_bytes / 2048)]
    # each probe twice (warm-up, timed); the timed one is summarised
    for c, n in lines.items():
        name = f"void (anonymous namespace)::k_probe_lines_coop<{c}u>(uint4 const*, unsigned long)"
        rows += [(name, 1, 1.0), (name, 1, n * 16 * c / 1024 / 2)]   # counter reads half: x2 scale
    for form, n in ((0, 1 << 27), (1, 1 << 27), (2, 1 << 27)):
        name = f"void (anonymous namespace)::k_probe_access<{form}u>(unsigned long*, unsigned long)"
        rows += [(name, 1, 1.0), (name, 1, n * 8 / 1024)]
    cas = "(anonymous namespace)::k_probe_cas(unsigned long*, unsigned long, unsigned long)"
    rows += [(cas, 1, 1.0), (cas, 1, (1 << 26) * 64 / 1024)]
    f = _db(tmp_path / "f.db", "FETCH_SIZE", rows)
    w = _db(tmp_path / "w.db", "WRITE_SIZE", [(COPY, 4096, copy_bytes / 1024)] + rows[1:])
    out = tmp_path / "p.json"
    ps.main(["probes", f, w, "--copy-bytes", str(copy_bytes), "--out", str(out)])
    r = json.loads(out.read_text())["per_access"]
    assert r["random_64B_line_read"]["fetch_bytes"] == 64.0
    assert r["random_128B_line_read"]["fetch_bytes"] == 128.0
    assert r["random_256B_line_read"]["fetch_bytes"] == 256.0
    assert r["slot_store_8B"]["fetch_bytes"] == 16.0 and r["slot_store_8B"]["write_bytes"] == 8.0
    assert r["cas_64bit"]["write_bytes"] == 64.0 and r["cas_64bit"]["accesses"] == 1 << 26


def test_traffic_sum_takes_per_kernel(tmp_path):
    copy_bytes = 1 << 20
    A = "void (anonymous namespace)::k_a<1, 8u>(int*)"
    Bk = "(anonymous namespace)::k_b(int*)"
    # two runs of [A, B, B], then more A and B work outside the runs
    runs = [(A, 1024, 5.0), (Bk, 1024, 1.0), (Bk, 1024, 2.0)] * 2 + [(A, 1024, 1000.0), (Bk, 1024, 1000.0)]
    f = _db(tmp_path / "f.db", "FETCH_SIZE", [(COPY, 4096, copy_bytes / 1024)] + runs)
    w = _db(tmp_path / "w.db", "WRITE_SIZE", [(COPY, 4096, copy_bytes / 1024)] + runs)
    out = tmp_path / "s.json"
    ps.main(["traffic-sum", f, w, "--kernel", "void k_a<1, 8u>", "--kernel", "k_b", "--take", "2", "--take", "4",
             "--runs", "2", "--units", "1", "--unit-name", "run", "--copy-bytes", str(copy_bytes), "--out", str(out)])
    r = json.loads(out.read_text())
    assert r["dispatches_per_run"] == 3
    assert r["fetch_bytes_per_run"] == (5.0 + 1.0 + 2.0) * 1024
