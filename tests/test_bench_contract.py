"""bench.py on the host: the one-GPU contract and the algorithmic byte
model behind roofline.achieved (no device needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line for a configuration it does not run


def test_algorithmic_bytes_model():
    import bench
    n = 1000
    # init + fix-up: 8(n+1) row_ptr + 8n parent/depth + 8n final pass
    base = 8 * (n + 1) + 8 * n + 8 * n
    assert bench.algorithmic_bytes([], n) == base
    td = {"direction": 1, "frontier": 10, "frontier_edges": 100, "claimed": 40,
          "scanned": 100, "unvisited": 0}
    # top-down: 20 per frontier vertex, 8 per frontier edge, 12 per claim
    assert bench.algorithmic_bytes([td], n) == base + 20 * 10 + 8 * 100 + 12 * 40
    bu = {"direction": 2, "frontier": 40, "frontier_edges": 400, "claimed": 300,
          "scanned": 900, "unvisited": 500}
    # switch to bottom-up: 4 per frontier vertex + n/8; then 16 per unvisited
    # vertex, 4 per scanned entry, three bitmaps, 8 per find
    want_bu = 4 * 40 + n // 8 + 16 * 500 + 4 * 900 + 3 * n // 8 + 8 * 300
    assert bench.algorithmic_bytes([td, bu], n) == base + 20 * 10 + 8 * 100 + 12 * 40 + want_bu
    # a second bottom-up level pays no conversion
    want_bu2 = 16 * 500 + 4 * 900 + 3 * n // 8 + 8 * 300
    assert bench.algorithmic_bytes([td, bu, bu], n) == (base + 20 * 10 + 8 * 100 + 12 * 40 + want_bu
                                                       + want_bu2)
    # back to top-down: the frontier bitmap becomes the queue (20 per
    # frontier vertex + n/8), then the top-down level itself
    td2 = {"direction": 1, "frontier": 30, "frontier_edges": 60, "claimed": 5,
           "scanned": 60, "unvisited": 0}
    want_td2 = 20 * 30 + n // 8 + 20 * 30 + 8 * 60 + 12 * 5
    assert bench.algorithmic_bytes([td, bu, td2], n) == (base + 20 * 10 + 8 * 100 + 12 * 40 + want_bu
                                                        + want_td2)


def test_batch_algorithmic_bytes_model():
    """The multi-source byte model, term by term (64 lanes: W = 1; 100
    lanes: W = 2)."""
    import bench
    n = 1000
    for lanes, W in ((64, 1), (100, 2)):
        base = 24 * W * n + 8 * lanes * n
        assert bench.batch_algorithmic_bytes([], n, lanes) == base
        td = {"direction": 1, "frontier": 10, "frontier_edges": 100, "claimed": 40,
              "scanned": 100, "unvisited": 0}
        want_td = 24 * W * n + 8 * W * 10 + 16 * 10 + 100 * (4 + 8 * W)
        assert bench.batch_algorithmic_bytes([td], n, lanes) == base + want_td
        bu = {"direction": 2, "frontier": 40, "frontier_edges": 400, "claimed": 300,
              "scanned": 900, "unvisited": 500}
        want_bu = 24 * W * n + 16 * 500 + 16 * W * 500 + 900 * (4 + 8 * W)
        assert bench.batch_algorithmic_bytes([td, bu], n, lanes) == base + want_td + want_bu


def test_level_attribution_matches_the_byte_model(tmp_path):
    """rocprof_summary levels: dispatches of the per-level schedule grouped
    into searches (statistics runs skipped), counters scaled by the copy
    kernel, and per-level algorithmic bytes that add up (with the
    initialisation and the final pass) to bench.algorithmic_bytes."""
    import csv
    import json
    import types
    import bench
    from paper_1508_03619_amd import rocprof_summary as rs
    n = 1000
    recs = [[1, 1, 5, 5, 5, 0], [1, 5, 40, 30, 40, 0], [2, 30, 500, 600, 900, 700],
            [2, 600, 100, 10, 12, 11], [1, 10, 20, 0, 20, 0]]
    as_dicts = [dict(zip(("direction", "frontier", "frontier_edges", "claimed", "scanned", "unvisited"), r))
                for r in recs]
    total = 16 * n + 8 + 8 * n
    prev = 1
    for r in recs:
        step, conv = rs.level_alg_bytes(r, prev, n)
        total += step + conv
        prev = r[0]
    assert total == bench.algorithmic_bytes(as_dicts, n)

    def rows(value):
        out, did = [], 0
        def emit(name, v, t=1000):
            nonlocal did
            did += 1
            out.append({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Value": v,
                        "Start_Timestamp": 0, "End_Timestamp": t})
        emit("gap::k_stream_copy(...)", 1024)
        for stats in (True, False):  # a statistics run, then the plain run
            emit("void gap::k_dd_init(gap::DDArgs*)", value)
            emit("void gap::k_dd_publish<%s>(gap::DDArgs*)" % str(stats).lower(), 0)
            for _ in recs:
                emit("void gap::k_dd_convert(gap::DDArgs*)", value)
                emit("void gap::k_dd_step<%s>(gap::DDArgs*)" % str(stats).lower(), value)
                emit("void gap::k_dd_publish<%s>(gap::DDArgs*)" % str(stats).lower(), 0)
            emit("void gap::k_dd_fixup(gap::DDArgs*)", value)
        return out

    for name, v in (("f.csv", 2), ("w.csv", 1)):
        with open(tmp_path / name, "w", newline="") as fh:
            w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Value",
                                               "Start_Timestamp", "End_Timestamp"])
            w.writeheader()
            w.writerows(rows(v))
    (tmp_path / "b.log").write_text("x\nLEVELS " + json.dumps({"graph": "g", "n": n, "source": 3,
                                                               "levels": recs}) + "\n")
    out = tmp_path / "o.txt"
    rs.levels(types.SimpleNamespace(fetch=str(tmp_path / "f.csv"), write=str(tmp_path / "w.csv"),
                                    log=str(tmp_path / "b.log"), out=str(out), copy_bytes=1024 * 8e6,
                                    cmd="test"))
    text = out.read_text()
    # copy kernel: 1024 units for 8.192e9 bytes -> 8e6 bytes per unit; a step
    # of 2 units fetched is 16 MB, of 1 unit written 8 MB
    line = [l for l in text.splitlines() if l.startswith("g bottom-up, first")][0].split()
    assert line[3:6] == ["1", "16.00", "8.00"], line  # one occurrence, MB fetched, MB written
    td = [l for l in text.splitlines() if l.startswith("g top-down, m_f <= 32768")][0].split()
    assert td[5] == "3", td  # three small top-down levels
    assert "g top-down, m_f <= 32768" in text and "g conversion" in text and "g final pass" in text
